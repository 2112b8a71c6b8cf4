/*
 * nfm.h -- C ABI of libnfm: multicanonical (MUCA) sampling of the 3D bimodal
 * Edwards-Anderson spin glass on one AMD Instinct MI355X (gfx950).
 *
 * Method: F. Muller, S. Schnabel, W. Janke, "Nonflat Histogram Techniques for
 * Spin Glasses" (arXiv:2011.08560).
 *   Model            Sec. II, Eq. (1): H = -sum_<ij> J_ij S_i S_j, S, J in {+1,-1},
 *                    simple-cubic lattice L^3 with periodic boundaries, 3V couplings
 *                    drawn +-1 with probability 1/2 and then quenched.
 *   Update           Sec. II, Eq. (2): single-spin Metropolis with acceptance
 *                    min(1, W(E_new)/W(E_old)) for energy weights W(E).
 *   Weights          Sec. II, Eqs. (3)-(7): flat W ~ 1/Omega, power law
 *                    W ~ P_SH/Omega with Eq. (5), 1/k-ensemble Eq. (7).
 *   Round trips      Sec. III: E ~ 0 -> lowest energy found -> E ~ 0.
 *
 * Conventions (all fixed by this header; every implementation must follow them):
 *   site           i = x + L*y + L*L*z, 0 <= x,y,z < L;
 *   couplings      3 planes of N = L^3 bits, plane d in {0:x,1:y,2:z}; bit i of
 *                  plane d is the bond between i and i+e_d; bit set <=> J = -1;
 *                  packed LSB-first into uint32 words, each plane padded to
 *                  JW = ceil(N/32) words (3*JW words per realization);
 *   spins          int8 +1/-1 per site at the ABI;
 *   energy levels  k = (E - e_base)/4, e_base = -3N + 2*(n_minus mod 2), where
 *                  n_minus is the number of J = -1 bonds; K = (3N - e_base)/4 + 1;
 *   sweep          N attempts in checkerboard order: every site with x+y+z even
 *                  (ascending i), then every odd one. Sweep t has attempt stamps
 *                  t*N + a + 1 for attempt a = 0..N-1;
 *   random words   Philox4x32-10 (Salmon et al., SC'11). The attempt at the q-th
 *                  site of colour c in plane z (q = y*L/2 + x/2) of sweep t, walker w
 *                  of realization id r uses output[q & 3] of counter
 *                  (((c*L + z) << 8) | (q >> 2), t, r, (w << 8) | 1) under
 *                  key = (walker_seed low, high) 32-bit halves;
 *   thresholds     a table row per level, 8 uint32 per row: entry u = 0..6 is the
 *                  acceptance threshold of a flip with u unsatisfied bonds
 *                  (Delta E = 12 - 4u); a move is accepted iff thr == 0xFFFFFFFF
 *                  or r < max(thr, 1) for the attempt's random word r (the least
 *                  probability of a move is 2^-32). A compact table
 *                  holds rows [row0, row0+rows); lookups clamp the level into it.
 *
 * Memory and streams: the caller owns all device memory. nfm_workspace_bytes()
 * returns the size of one device buffer; the caller allocates it (e.g. a torch
 * tensor) and passes its address to nfm_create(). Every kernel of a context is
 * launched on the HIP stream given at creation. Host arrays passed to the API
 * are borrowed for the duration of the call only. Functions named nfm_get_* /
 * nfm_read_* synchronize the stream; the others are asynchronous unless stated.
 *
 * Errors: every function returns an nfm_status. Invalid arguments return
 * NFM_EINVAL and change no state; nfm_last_error() describes the last failure.
 * No C++ exception crosses this boundary.
 */
#ifndef NFM_H
#define NFM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NFM_OK = 0,
  NFM_EINVAL = -1,   /* invalid argument (unsupported L, bad range, null pointer) */
  NFM_ERANGE = -2,   /* value out of the representable range (sweep counter, sizes) */
  NFM_EDEVICE = -3,  /* HIP runtime error */
  NFM_ESTATE = -4,   /* call not valid in the current state */
  NFM_ESIZE = -5     /* workspace too small */
} nfm_status;

typedef struct nfm_ctx nfm_ctx;

/* Batch description. All realizations of a context share the seeds; realization
 * r (0-based in the batch) has id first_real_id + r in the random streams. */
typedef struct {
  int32_t n_real;            /* realizations in the batch, >= 1 */
  const int32_t* L;          /* host [n_real]: linear size; even, 2 <= L <= 12 */
  const int32_t* walkers;    /* host [n_real]: walkers per realization, multiple of 64 */
  uint64_t disorder_seed;    /* Philox key of the couplings */
  uint64_t walker_seed;      /* Philox key of initial spins and acceptance words */
  uint32_t first_real_id;
  int32_t trace_capacity;    /* sweeps of per-walker energy trace kept (0 = none) */
} nfm_batch_desc;

/* Per-walker state as read back (host layout, 40 bytes). */
typedef struct {
  int32_t E;          /* current energy */
  int32_t E_min;      /* lowest energy seen */
  int32_t rt_state;   /* 0: top not reached yet, 1: at/after top, 2: bottom after top */
  int32_t new_min;    /* 1 once an energy below e_bot was seen (sample must be rerun) */
  uint64_t rt_count;  /* completed round trips */
  uint64_t t_first;   /* attempt stamp of the first arrival at the top */
  uint64_t t_last;    /* attempt stamp of the last completed round trip */
} nfm_walker_stats;

/* Per-realization integer sums over its walkers (host layout, 40 bytes). */
typedef struct {
  uint64_t rt_count;  /* sum of rt_count */
  uint64_t rt_time;   /* sum over walkers with rt_count > 0 of (t_last - t_first), attempts */
  int32_t E_min;      /* minimum of E_min */
  int32_t new_min;    /* OR of new_min */
  int32_t walkers_with_trips;
  int32_t pad;
  uint64_t reserved;
} nfm_real_stats;

/* Size of the device workspace for a batch. Sec. II (model sizes). */
nfm_status nfm_workspace_bytes(const nfm_batch_desc* desc, size_t* bytes);

/* Create a context over a caller-owned device workspace of at least
 * nfm_workspace_bytes() bytes (256-byte aligned) on device `device`, launching on
 * `hip_stream` (a hipStream_t; NULL = default stream). The workspace is not freed
 * by the library. */
nfm_status nfm_create(nfm_ctx** out, const nfm_batch_desc* desc, void* dev_workspace,
                      size_t workspace_bytes, int device, void* hip_stream);
/* Waits for the context's stream, then frees the context's host-side state (NULL is a no-op);
 * the device workspace stays the caller's. */
void nfm_destroy(nfm_ctx* ctx);
/* Message of the context's last failed call; owned by the context, valid until its next call. */
const char* nfm_last_error(const nfm_ctx* ctx);

/* Geometry queries (host-side, no synchronization). */
int32_t nfm_n_real(const nfm_ctx* ctx);
int64_t nfm_n_walkers(const nfm_ctx* ctx);              /* total walkers of the batch */
int32_t nfm_levels(const nfm_ctx* ctx, int32_t r);      /* K of realization r (after couplings) */
int32_t nfm_e_base(const nfm_ctx* ctx, int32_t r);      /* e_base of realization r */
int64_t nfm_level_offset(const nfm_ctx* ctx, int32_t r);/* start of r in histogram / level arrays */
int64_t nfm_levels_total(const nfm_ctx* ctx);           /* length of histogram / level arrays */
int64_t nfm_walker_offset(const nfm_ctx* ctx, int32_t r);/* global index of r's first walker */
uint64_t nfm_sweep_counter(const nfm_ctx* ctx);         /* sweeps done so far */

/* Couplings. Sec. II: 3V couplings +-1 with p = 1/2, drawn once per realization.
 * nfm_init_couplings draws them on the device: bit c (c = d*N + i) is bit c%32 of
 * output[m & 3] of counter (m >> 2, id, 0, 3), m = c/32, key = disorder_seed.
 * nfm_set_couplings / nfm_get_couplings copy realizations [r0, r0+count) in the
 * ABI layout (3*JW words each, host). Setting couplings resets the energy levels,
 * tables and histograms of those realizations; call nfm_compute_energies after
 * changing spins or couplings. */
nfm_status nfm_init_couplings(nfm_ctx* ctx);
nfm_status nfm_set_couplings(nfm_ctx* ctx, int32_t r0, int32_t count, const uint32_t* host_words);
nfm_status nfm_get_couplings(nfm_ctx* ctx, int32_t r0, int32_t count, uint32_t* host_words);

/* Spins. nfm_init_spins draws every walker's start: bit i is bit i%32 of
 * output[m & 3] of counter (m >> 2, 0, id, (w << 8) | 2), m = i/32, key =
 * walker_seed; set bit <=> S = -1. Set/get copy walkers [w0, w0+count) (global
 * walker index; realization r owns [nfm_walker_offset(r), +walkers[r])), N int8 each, back
 * to back (a range may span realizations of different L: each walker takes its own N). */
nfm_status nfm_init_spins(nfm_ctx* ctx);
nfm_status nfm_set_spins(nfm_ctx* ctx, int64_t w0, int64_t count, const int8_t* host_spins);
nfm_status nfm_get_spins(nfm_ctx* ctx, int64_t w0, int64_t count, int8_t* host_spins);

/* Eq. (1) for every walker; resets E_min = E, round-trip state, counters and
 * new_min of every walker. */
nfm_status nfm_compute_energies(nfm_ctx* ctx);

/* Tables. nfm_set_thresholds copies a raw table for realization r: rows x 8
 * uint32 (host) covering levels [row0, row0+rows); 1 <= rows <= K.
 * nfm_set_weights_lnw builds the tables of all realizations on the device from
 * log-weights: host lnw holds nfm_levels_total() doubles, realization r's level k
 * at index nfm_level_offset(r) + k (only [k_lo[r], k_top[r]] is read); the table covers
 * [max(0,k_lo-3), min(K-1,k_top+3)] with step log-weights d(j) = lnw(j+1)-lnw(j)
 * on [k_lo, k_top), d(j) = 0 for j >= k_top, d(j) = d(k_lo) for j < k_lo; entry
 * (k,u), m = 3-u: x = exp(d(k)+..+d(k+m-1)) (m>0), exp(-(d(k+m)+..+d(k-1))) (m<0),
 * 1 (m=0), sums in ascending j; thr = 0xFFFFFFFF if x >= 1 else floor(x*2^32).
 * Eq. (2) with weights from Eqs. (3)-(7). */
nfm_status nfm_set_thresholds(nfm_ctx* ctx, int32_t r, const uint32_t* host_thr, int32_t row0,
                              int32_t rows);
nfm_status nfm_get_thresholds(nfm_ctx* ctx, int32_t r, uint32_t* host_thr, int32_t* row0,
                              int32_t* rows);
nfm_status nfm_set_weights_lnw(nfm_ctx* ctx, const double* host_lnw, const int32_t* k_lo,
                               const int32_t* k_top);

/* Round-trip bounds of realization r (Sec. III): the top is E >= e_top, the bottom
 * E <= e_bot; an energy below e_bot sets new_min. Default: e_top = 0 and
 * e_bot = e_base - 4 (no bottom). Takes effect at the next nfm_run_sweeps. */
nfm_status nfm_set_rt_bounds(nfm_ctx* ctx, int32_t r, int32_t e_bot, int32_t e_top);

/* Run n_sweeps sweeps of every walker (asynchronous). After every attempt the
 * walker's minimum and round-trip state are updated (stamp t*N + a + 1); after
 * every sweep its level is added to its realization's histogram and its energy
 * to its trace (while fewer than trace_capacity sweeps have been traced since
 * the last nfm_reset_trace). Sec. II, Eq. (2); Sec. III. n_sweeps = 0 changes no state.
 * NFM_ESTATE before couplings and every realization's table are set; NFM_ERANGE when the
 * context's sweep counter would pass 2^32 - 1 (the sweep index is one word of the random
 * stream's counter). */
nfm_status nfm_run_sweeps(nfm_ctx* ctx, uint64_t n_sweeps);

/* Histograms: nfm_levels_total() uint64; realization r's count of level k is at
 * nfm_level_offset(r) + k (each realization reserves 3N/2+1 entries, K of them used).
 * Counts accumulate since the last reset; reset != 0 clears them after reading. */
nfm_status nfm_read_histograms(nfm_ctx* ctx, uint64_t* host_dst, int reset);
nfm_status nfm_reset_histograms(nfm_ctx* ctx);
nfm_status nfm_read_walkers(nfm_ctx* ctx, nfm_walker_stats* host_dst);   /* all walkers */
nfm_status nfm_read_realizations(nfm_ctx* ctx, nfm_real_stats* host_dst); /* all realizations */
/* Trace: the traced walkers x capacity int32 (walker-major); entry s of a walker is its energy
 * after the s-th traced sweep; *n_valid receives the number of traced sweeps. By default every
 * walker of the batch is traced with capacity = the description's trace_capacity.
 * nfm_reset_trace restarts the trace at the current sweep.
 * nfm_trace_config traces the walkers [walker_begin, walker_begin + count) (global indices) for up
 * to `capacity` sweeps each, from the current sweep on (Sec. III's energy traces of chosen
 * walkers at a longer horizon): NFM_EINVAL unless the range lies in the batch and capacity >= 0,
 * NFM_ESIZE if count x capacity exceeds the trace region the workspace holds (all walkers x
 * trace_capacity). nfm_read_trace then copies count x capacity entries. Checkpoints keep it. */
nfm_status nfm_read_trace(nfm_ctx* ctx, int32_t* host_dst, int32_t* n_valid);
nfm_status nfm_reset_trace(nfm_ctx* ctx);
nfm_status nfm_trace_config(nfm_ctx* ctx, int64_t walker_begin, int64_t count, int32_t capacity);
/* The traced range and capacity in effect (host-side, no synchronization). */
nfm_status nfm_trace_range(const nfm_ctx* ctx, int64_t* walker_begin, int64_t* count, int32_t* capacity);

/* Inject histograms (nfm_levels_total() uint64, same layout as nfm_read_histograms). */
nfm_status nfm_set_histograms(nfm_ctx* ctx, const uint64_t* host_src);
/* Clear every walker's round-trip state, counters and new_min (E and E_min kept), e.g. before
 * a production run (Sec. III: round trips are counted in production). */
nfm_status nfm_reset_round_trips(nfm_ctx* ctx);
/* Stuck-walker watch (failure detection; no passage of the paper defines it: Sec. III counts
 * round trips between the energy bounds, and a walker that stops completing them holds up its
 * sample's requeue for 100 trips). Flags every walker whose last completed round trip lies
 * window_sweeps or more sweeps before the context's sweep counter; a walker without one counts
 * from the sweep at which its round-trip state was last cleared (nfm_compute_energies,
 * nfm_reset_round_trips). Age in whole sweeps = floor((sweeps * N - t_last) / N), t_last in
 * attempt stamps. device_flags: NULL or a device buffer of nfm_n_walkers() bytes (1 flagged,
 * 0 not; written on the context's stream); *host_count: the number flagged (the call waits for
 * the stream). window_sweeps = 0 flags every walker. EINVAL on a null count. */
nfm_status nfm_stuck_walkers(nfm_ctx* ctx, uint64_t window_sweeps, uint8_t* device_flags, int64_t* host_count);

/* Weight iteration on the device (Sec. II: the DOS estimate is iterated once per realization,
 * with power-law shaped targets, and reused by every ensemble). Profiles: 0 flat (Eq. (3)),
 * 1 power law (Eqs. (4), (5): ln P = alpha ln((E - E_g + dE)/(dE - E_g)), E_g the lowest energy
 * found; dE > 0, alpha <= 0), 2 the 1/k-ensemble (Eq. (7)).
 * State per realization: DOS steps b(k) = S(k+1) - S(k) and their accumulated weights p(k)
 * (FP64, nfm_level_offset layout), visited levels, k_lo (lowest level found), k_top (lowest
 * level with E >= 0). Weights lnW = -S + ln P on [k_lo, k_top] with S(k_top) = 0.
 *
 * nfm_rec_init: b = p = 0, k_lo from the walkers' minima; builds weights and tables, sets the
 *   round-trip bounds to e_bot = E(k_lo), e_top = 0, clears the histograms.
 * nfm_rec_update: one update from the histograms accumulated since the last init/update
 *   (synchronizes): k_lo <- min(k_lo, walkers' minima) (new levels take b(k_lo), p = 0); for
 *   consecutive visited levels k < k': est = [ln H(k') - lnW(k')] - [ln H(k) - lnW(k)] (lnW
 *   continued below the old k_lo with its lowest step), g0 = H(k)H(k')/(H(k)+H(k')), p(k) += g0,
 *   b(k) += (g0/p(k)) (est - (b(k)+...+b(k'-1))); flatness = min/mean of H/P over levels ever
 *   visited in [k_lo, k_top]; converged iff flatness >= f_tol and k_lo unchanged. Then the next
 *   weights (profile re-anchored at the new k_lo), tables and bounds; histograms cleared.
 *   host_info (optional) receives every realization's nfm_rec_info.
 * nfm_rec_production: tables from the current estimate with the given profile (flat lnW = -S,
 *   power law -S + ln P, 1/k -ln sum_{j<=k} exp S), bounds e_bot = E(k_lo), e_top = 0,
 *   histograms cleared. */
typedef struct {
  int32_t k_lo, k_top;
  int32_t profile;
  int32_t converged;     /* last update: flat to f_tol and no new minimum */
  int32_t iterations;    /* updates done */
  int32_t k_lo_changed;  /* last update lowered k_lo */
  double pl_dE, pl_alpha;
  double flatness;       /* last update */
  int32_t k_seed;        /* -1, or the lowest level of a seeded prior (nfm_rec_seed) */
  int32_t pad;
} nfm_rec_info;

nfm_status nfm_rec_init(nfm_ctx* ctx, int32_t profile, double pl_dE, double pl_alpha);
nfm_status nfm_rec_update(nfm_ctx* ctx, double f_tol, nfm_rec_info* host_info);
nfm_status nfm_rec_production(nfm_ctx* ctx, int32_t profile, double pl_dE, double pl_alpha);
nfm_status nfm_rec_read_info(nfm_ctx* ctx, nfm_rec_info* host_info);
/* Read / write one realization's recursion state (arrays of 3N/2+1 entries; any pointer of
 * rec_get_state may be NULL). rec_set_state also marks the recursion as initialized. */
nfm_status nfm_rec_get_state(nfm_ctx* ctx, int32_t r, double* b, double* p, double* S, double* lnP,
                             double* lnW, uint8_t* visited, nfm_rec_info* info);
nfm_status nfm_rec_set_state(nfm_ctx* ctx, int32_t r, const double* b, const double* p,
                             const double* lnP, const double* lnW, const uint8_t* visited,
                             const nfm_rec_info* info);

/* Wang-Landau estimate of the density of states (named in Sec. II as an alternative estimator;
 * its steps are not printed there), in batched form: the walkers of a realization share one
 * estimate ln g on the levels [0, k_top] (k_top = lowest level with E >= 0; W constant above).
 * nfm_wl_init: ln g = 0, ln f = ln_f0 > 0, stage histogram 0, weights lnW = -ln g = 0 and their
 *   tables (rows from level 0 to k_top + 3); clears the histograms.
 * A step: nfm_run_sweeps(n), then nfm_wl_update: every level k <= k_top gains
 *   ln g(k) += ln f H(k) (H = the histogram since the last update, one entry per walker per
 *   sweep), H is added to the stage histogram Hs and cleared; flatness = min/mean of Hs over the
 *   levels it visited; if flatness >= flat_tol, ln f <- ln f / 2 (a new stage, Hs cleared) and the
 *   realization is done once ln f < ln_f_final (later updates leave it unchanged). Then the next
 *   weights and tables. host_info (may be NULL) receives every realization's nfm_wl_info.
 * nfm_wl_get: realization r's ln g and stage histogram (3N/2+1 entries each; either may be NULL).
 * nfm_wl_to_rec: hands the estimate to the recursion (nfm_rec_*): visited = levels with ln g > 0,
 *   k_lo the lowest of them, b(k) = ln g(k+1) - ln g(k) on [k_lo, k_top), p = 0, the given
 *   profile; weights, tables and round-trip bounds as after nfm_rec_update; clears the
 *   histograms. The recursion can then refine it (nfm_rec_update) or produce (nfm_rec_production). */
typedef struct {
  double ln_f;       /* current modification factor */
  double flatness;   /* last update */
  int32_t stage;     /* halvings so far */
  int32_t done;      /* ln f < ln_f_final */
  int32_t k_top;
  int32_t updates;
} nfm_wl_info;
nfm_status nfm_wl_init(nfm_ctx* ctx, double ln_f0);
nfm_status nfm_wl_update(nfm_ctx* ctx, double flat_tol, double ln_f_final, nfm_wl_info* host_info);
nfm_status nfm_wl_get(nfm_ctx* ctx, int32_t r, double* host_lng, uint64_t* host_hst, nfm_wl_info* info);
nfm_status nfm_wl_to_rec(nfm_ctx* ctx, int32_t profile, double pl_dE, double pl_alpha);

/* Launch tuning of nfm_run_sweeps (results do not depend on it: the random stream is indexed
 * by sweep, site and walker, and all accumulation is integer).
 *   speculate: -1 automatic (= off), 0 off, 1 on. With speculation each attempt also loads the
 *     next site's two candidate thresholds (accepted / rejected) before its own decision
 *     resolves, which shortens a walker's serial chain at the cost of a second table read. The
 *     plain form overlaps its single table read with generator work instead, which measures
 *     faster on gfx950 at every occupancy tried.
 *   sweeps_per_launch: sweeps per kernel launch, at most 2^20 (0 = 1024). A launch keeps its
 *     walkers' histogram counts on chip and adds them to the histograms when it ends.
 *   schedule: 0 = one launch per lattice size of the batch; 1 = one persistent launch for the
 *     whole batch, whose workgroups take waves of walkers from a queue ordered by decreasing N
 *     (longest first), so that realizations of uneven size share the GPU; 2 = split: the
 *     largest size's waves as a persistent queue of their own in a kernel form whose waves each
 *     hold a whole SIMD (their serial chains bound a sweep of the batch, and run fastest alone),
 *     beside a persistent queue over the remaining sizes on the SIMDs left free (at most half the
 *     SIMDs go to the largest size), launched on a second stream of the library's behind a short
 *     wait, forked from and joined to the context's stream; a batch of one size runs as 1. A
 *     persistent launch over sizes up to 8 or 10 uses the form compiled for them (fewer registers).
 *   waves_per_cu: persistent schedule only, resident workgroups per compute unit (0 = as many
 *     as fit).
 *   hist: extent of a launch's on-chip histogram. 0 automatic: every level of the realization
 *     when that leaves as many workgroups resident per compute unit as the window (capped at the
 *     ones the launch needs), else the window; 1 window: the table's rows and 64 levels on either
 *     side, levels outside it counted in device memory directly; 2 every level; 3 the table's
 *     rows alone (the most direct counting; for tests of that path).
 *   ws: per-size launches with the expanded table only: a second wave per workgroup computes the
 *     sampling wave's random words into LDS, two plane blocks ahead (the same words, so the same
 *     results). 0 automatic: when the launch has at most one wave of walkers per SIMD and all its
 *     workgroups fit at once; 1 never; 2 always. */
typedef struct {
  int32_t speculate;
  int32_t sweeps_per_launch;
  int32_t schedule;
  int32_t waves_per_cu;
  int32_t hist;
  int32_t ws;
} nfm_tuning;
nfm_status nfm_set_tuning(nfm_ctx* ctx, const nfm_tuning* tuning);
nfm_status nfm_get_tuning(const nfm_ctx* ctx, nfm_tuning* tuning);

/* Autotuner for mixed batches (no passage of the paper: a launch-configuration search). Times
 * every candidate tuning (speculation off/on x sweeps per launch {16, 64, 256, 1024} x {per-size
 * launches without and (no speculation) with the generator wave, persistent queue with as many
 * workgroups as fit, 4 or 8 per CU, split}, and at 256 sweeps per launch the two persistent forms
 * with the histogram as the window alone instead of automatic) for calib_sweeps
 * sweeps on the batch itself, then restores spins, walker state and histograms, so the
 * calibration leaves no trace in the results (the sweep counter does not move). The fastest
 * candidate (spin-flip attempts per second) is applied and returned in *best. Results are cached
 * per (device, CU count, mix of L and walkers) for the process and, when cache_path is not
 * NULL, in that text file (one line per key; a cached key is applied without measuring, and
 * *n_results is then 0). results may be NULL when max_results is 0. Needs couplings and tables. */
typedef struct {
  nfm_tuning tuning;
  double attempts_per_s;
} nfm_tune_result;
nfm_status nfm_autotune(nfm_ctx* ctx, int32_t calib_sweeps, const char* cache_path, nfm_tune_result* results,
                        int32_t max_results, int32_t* n_results, nfm_tuning* best);

/* Waits for every launch on the context's stream; NFM_EDEVICE reports a device error raised by
 * an earlier asynchronous call. */
nfm_status nfm_sync(nfm_ctx* ctx);
/* Name of the sweep kernel form the last sweep launch on the calling host thread used, e.g.
 * "k_sweeps_ws<6>" (a report for benchmarks; "none" before any launch). */
const char* nfm_last_kernel(const nfm_ctx* ctx);

/* Checkpoint and resume (the sweep counter travels with the state, so a run resumed from a
 * checkpoint draws the same random words and gives the same spins, energies, histograms, round
 * trips, traces, weights and tempering state as the run that was never interrupted).
 * nfm_checkpoint_bytes: size of a checkpoint of this context (a header, the host-side scalars
 *   and tempering temperatures, and a byte copy of the whole workspace).
 * nfm_checkpoint: waits for all work queued on the stream, then writes the checkpoint into the
 *   caller's host buffer of `capacity` bytes (NFM_ESIZE if smaller than nfm_checkpoint_bytes).
 * nfm_restore: loads a checkpoint into a context created from the same batch description (sizes,
 *   walkers, realization ids, seeds, trace capacity; NFM_EINVAL otherwise, NFM_ESIZE if
 *   truncated), replacing its whole state, tuning included. The workspace may sit at another
 *   device address or on another context of the same description. Synchronizes. */
nfm_status nfm_checkpoint_bytes(const nfm_ctx* ctx, size_t* bytes);
nfm_status nfm_checkpoint(nfm_ctx* ctx, void* host_blob, size_t capacity);
nfm_status nfm_restore(nfm_ctx* ctx, const void* host_blob, size_t size);

/* ---------------------------------------------------------------------------------------
 * Parallel tempering (Sec. II, Eq. (8)), the baseline the paper compares against. Each group
 * of 64 walkers of a realization (walkers 64q .. 64q + 63) holds floor(64/M) sets of M
 * configurations: set g of the group is walkers 64q + gM + c, c = 0..M-1, with set index
 * q floor(64/M) + g within the realization; the group's remaining walkers idle at slot 0 (they
 * sweep at the lowest temperature and take part in no exchange and no round-trip bookkeeping).
 * Each configuration sits at one temperature slot of its set, slots being a permutation of
 * 0..M-1. Temperatures T_0 < ... < T_{M-1} are per realization. One PT sweep: every
 * configuration makes one checkerboard sweep of canonical Metropolis attempts at its slot's
 * temperature (random words as in nfm_run_sweeps, tag 4 instead of 1); then its energy goes
 * through the round-trip bookkeeping (bounds of nfm_set_rt_bounds; stamp (t+1) N, so round-trip
 * times come out in PT sweeps) and the trace; then the slot pairs (s, s+1) with s = t (mod 2)
 * try an exchange with probability min(1, exp((1/T_{s+1} - 1/T_s)(E_{s+1} - E_s))), taking
 * output[s & 3] of Philox counter (s >> 2, t, real_id, (set << 8) | 5) under the walker seed.
 * Thresholds, with beta = 1.0/T in FP64: Metropolis entry u of slot s, floor(exp(-beta_s 4m) 2^32)
 * for m = 3 - u > 0 and 0xFFFFFFFF for m <= 0 (acceptance as in nfm_run_sweeps), computed on the
 * host whenever temperatures change; exchange of slots (s, s+1) whose energies differ by 4d,
 * d > 0: floor(q_s^d 2^32) (0xFFFFFFFF if q_s^d >= 1) with q_s = exp(4 (beta_{s+1} - beta_s))
 * from the host and q_s^d formed on the device by binary powering (r = 1, b = q; per bit of d
 * from the lowest: r *= b if set, then b *= b; FP64 products), accepted iff it is 0xFFFFFFFF or
 * r < it. The power has no cap on d.
 * Energies are tracked per attempt, so nfm_compute_energies must have run first.
 *
 * nfm_pt_init: M in [2, 64]; host_temps[M] strictly increasing, > 0, for every realization;
 *   puts configuration c of every set at slot c (idle walkers at 0) and clears the exchange
 *   counters. Round-trip state is left as is (see nfm_reset_round_trips). EINVAL on bad M or
 *   temperatures, ESTATE without couplings.
 * nfm_pt_set_temps / nfm_pt_get_temps: the M temperatures of realization r.
 * nfm_pt_get_tables: the thresholds the kernel uses for realization r, for inspection: metro
 *   [M][8] (u-order, entry 7 = 0), swap [M-1][D] for d = 1..D with D the first d at which every
 *   pair's threshold is 0 (at most 3N/2 + 1 of the largest N); either array may be NULL.
 * nfm_pt_adapt: one step of the per-realization temperature adaptation for a constant exchange
 *   rate (the paper's protocol, Sec. II; its rule is not printed, this is a reading): from the
 *   exchanges accepted since the last adapt (or init), the rate A_s of each pair of each
 *   realization (over its sets and the sweeps that attempted the pair); host_rates (may be NULL)
 *   receives them, [n_real][M-1], and *n_outside (may be NULL) the number outside
 *   [rate_lo, rate_hi]. Then every gap beta_s - beta_{s+1} is multiplied by (-ln A_s)^(-1/4)
 *   (A_s clamped to [1e-6, 1 - 1e-12]; half the step that equalises A = exp(-c gap^2)), that
 *   factor limited to [1/2, 2], and the gaps are rescaled to their old sum, keeping T_0 and
 *   T_{M-1}; counters cleared.
 *   ESTATE before two PT sweeps since the last clear. */
nfm_status nfm_pt_init(nfm_ctx* ctx, int32_t M, const double* host_temps);
nfm_status nfm_pt_set_temps(nfm_ctx* ctx, int32_t r, const double* host_temps);
nfm_status nfm_pt_get_temps(nfm_ctx* ctx, int32_t r, double* host_temps);
nfm_status nfm_pt_get_tables(nfm_ctx* ctx, int32_t r, uint32_t* host_metro, uint32_t* host_swap, int32_t* M,
                             int32_t* D);
nfm_status nfm_pt_adapt(nfm_ctx* ctx, double rate_lo, double rate_hi, double* host_rates, int32_t* n_outside);
/* Run n PT sweeps of every walker (asynchronous on the stream; advances the sweep counter). */
nfm_status nfm_pt_run_sweeps(nfm_ctx* ctx, uint64_t n_sweeps);
/* Slots of all walkers (int32, nfm_n_walkers() entries); set_slots checks that each set holds a
 * permutation of 0..M-1 and that idle walkers are at slot 0. */
nfm_status nfm_pt_read_slots(nfm_ctx* ctx, int32_t* host_slots);
nfm_status nfm_pt_set_slots(nfm_ctx* ctx, const int32_t* host_slots);
/* Accepted exchanges since nfm_pt_init or the last nfm_pt_adapt: uint64 [n_sets][M - 1], sets in
 * walker order (realization by realization, set index within it), entry [g][s] for the pair
 * (s, s+1). n_sets = (n_walkers / 64) floor(64/M). */
nfm_status nfm_pt_read_exchanges(nfm_ctx* ctx, uint64_t* host_acc);

/* ---------------------------------------------------------------------------------------
 * Round-trip statistics (Sec. III). For realization r: tau_r = (sum over walkers with trips of
 * t_last - t_first) / (trips) / N, in sweeps (the stamps count attempts), NaN when it has fewer
 * than max(1, min_trips) trips (censored). tau_pop = mean of the uncensored tau_r of the range.
 * host_tau (may be NULL) receives count doubles. Synchronizes. */
typedef struct {
  double tau_pop;      /* NaN if every realization of the range is censored */
  uint64_t trips;      /* completed round trips in the range */
  int32_t n_used;      /* uncensored realizations */
  int32_t n_censored;
} nfm_rt_summary;
nfm_status nfm_rt_stats(nfm_ctx* ctx, int32_t r0, int32_t count, uint64_t min_trips, double* host_tau,
                        nfm_rt_summary* host_summary);

/* ---------------------------------------------------------------------------------------
 * Round-trip-time statistics across realizations (Secs. IV and V). Host functions, no context, no
 * device: inputs are per-realization mean round-trip times (nfm_rt_stats), all finite and > 0.
 *
 * Frechet distribution, Eq. (9): F(tau) = exp(-(1 + xi (tau - mu)/beta)^(-1/xi)) on
 * tau >= mu - beta/xi, with beta > 0, xi > 0.
 *   nfm_frechet_cdf: F(tau) (0 below the support).
 *   nfm_frechet_quantile: Q(p), Eq. (13), p in (0, 1) (NaN outside).
 *   nfm_frechet_mean: Eq. (11), mu + beta/xi (Gamma(1 - xi) - 1) for xi < 1, +inf otherwise.
 *   nfm_frechet_quantile_mean: Eq. (14), the mean integral cut at Q(1 - eps) and not renormalized,
 *     in closed form (mu - beta/xi)(1 - eps) + beta/xi Gamma(1 - xi, -ln(1 - eps)); eps in [0, 1)
 *     (eps = 0 gives Eq. (11)). For xi < 0.01, where the two terms cancel, the same value as
 *     mu (1 - eps) + beta int_x^inf (t^-xi - 1)/xi e^-t dt, x = -ln(1 - eps) (quadrature).
 *   nfm_upper_gamma: the upper incomplete gamma function Gamma(a, x) for real a and x > 0 (NaN
 *     otherwise); for a <= 0 by Gamma(a, x) = (Gamma(a + 1, x) - x^a e^-x) / a from (0, 1], or
 *     from E1 = Gamma(0, x).
 *   nfm_frechet_fit: the parameters fitted to n >= 3 times (the paper fits "the CDF" without
 *     naming the estimator): method 0 = maximum likelihood, 1 = least squares between F and the
 *     plotting positions (i - 1/2)/n of the sorted times. *objective (may be NULL) receives the
 *     minimised negative log-likelihood or sum of squares. NFM_EINVAL for bad input (message in
 *     nfm_stats_last_error()).
 *   nfm_relative_performance: r of Table I for paired samples (index i = the same disorder
 *     realization under both methods): r_pop = mean(tau_m) / mean(tau_ref) and
 *     r_eps = <tau>_eps(fit of tau_m) / <tau>_eps(fit of tau_ref), each with a jackknife error
 *     from `blocks` contiguous blocks of realizations left out in turn (0 = one realization per
 *     block); also the two full-sample fits. eps in (0, 1). */
typedef struct {
  double mu, beta, xi;
} nfm_frechet;
typedef struct {
  double r_pop, r_pop_err, r_eps, r_eps_err;
  nfm_frechet fit_m, fit_ref;
  int32_t blocks, pad;
} nfm_ratio;
double nfm_frechet_cdf(const nfm_frechet* d, double tau);
double nfm_frechet_quantile(const nfm_frechet* d, double p);
double nfm_frechet_mean(const nfm_frechet* d);
double nfm_frechet_quantile_mean(const nfm_frechet* d, double eps);
double nfm_upper_gamma(double a, double x);
nfm_status nfm_frechet_fit(const double* tau, int64_t n, int32_t method, nfm_frechet* fit, double* objective);
nfm_status nfm_relative_performance(const double* tau_m, const double* tau_ref, int64_t n, double eps,
                                    int32_t method, int32_t blocks, nfm_ratio* out);
/* nfm_frechet_fit_jackknife: the fit of nfm_frechet_fit to n >= 3 times and the delete-a-block
 *   jackknife errors of (mu, beta, xi): the fit is repeated with each of B contiguous blocks
 *   [b n / B, (b + 1) n / B) left out (B = n for blocks = 0, else blocks in [2, n], every subsample
 *   keeping at least 3 times) and err^2 = (B - 1)/B sum_b (theta_b - mean theta)^2 per parameter
 *   (Sec. IV: Fig. 4 plots the shape xi per size and method with such errors). *blocks_used (may
 *   be NULL) receives B.
 * nfm_running_mean: out[i] = (tau_0 + ... + tau_i) / (i + 1), the running mean of Eq. (12) (Sec. V,
 *   plotted in Fig. 5) over the realizations in the given order, summed left to right.
 * nfm_frechet_ks: sup over tau of |F_n(tau) - F(tau)| between the empirical CDF of the n times
 *   and Eq. (9) with the given parameters (the fit quality behind Fig. 3), evaluated at the sorted
 *   times from both sides of each step. */
nfm_status nfm_frechet_fit_jackknife(const double* tau, int64_t n, int32_t method, int32_t blocks, nfm_frechet* fit,
                                     nfm_frechet* err, int32_t* blocks_used);
nfm_status nfm_running_mean(const double* tau, int64_t n, double* out);
nfm_status nfm_frechet_ks(const nfm_frechet* d, const double* tau, int64_t n, double* dist);
/* Message of the calling thread's last failed statistics call (thread-local storage). */
const char* nfm_stats_last_error(void);

/* ---------------------------------------------------------------------------------------
 * Learned start of the weight iteration (not in the paper: a model that guesses the density of
 * states from the couplings, checked by the recursion of Sec. II, which decides the final estimate).
 *
 * nfm_set_canonical: canonical Metropolis tables at temperature T > 0 for every realization
 *   (lnW = -E/T; the two top levels are given and the lowest step continues below, which is
 *   the same constant step), for the short run whose histogram feeds the model.
 * nfm_features: dev_x (device, n_real x 81 floats) receives per realization: L/12; the
 *   frustrated fraction of (x,y), (y,z), (z,x) plaquettes and of all (a plaquette (i; d1, d2)
 *   has bonds J_d1(i), J_d2(i+e_d1), J_d1(i+e_d2), J_d2(i), frustrated when their product is
 *   -1); the negative-bond fraction along x, y, z and of all bonds; n_minus mod 2; the fraction
 *   of elementary cubes with 0, 2, 4, 6 frustrated faces; mean/6, variance/6 and fourth central
 *   moment/96 of the site sums sum_j J_ij; then 64 bins of E/N over [-2, 0) (bin
 *   floor((E/N + 2) 32) clipped to [0, 63]) of the current level histogram, as fractions.
 * nfm_rec_seed: a seeded prior on the DOS steps. For realization r with host_k_seed[r] >= 0
 *   (and < k_top): b(k) = host_b[level offset + k] on [k_seed, k_top), accumulated weights p
 *   cleared. A seeded estimate continues S below k_lo with its own steps (profile frozen at
 *   k_lo), so weights and tables cover [min(k_seed, k_lo), k_top], and levels reached for the
 *   first time keep their seeded steps (unseeded: they copy the lowest known step). k_lo still
 *   comes from the walkers, and round trips, flatness and convergence are defined as before.
 *   Weights, tables and bounds are rebuilt. Needs nfm_rec_init. host_k_seed = -1: unchanged.
 * nfm_rec_seed_grid: the same from curves y (device, n_real x 256 floats) with y_j = [S(E) -
 *   S(E_top)]/N on e_j = -2 + 2j/255: S(k) = N y(E_k/N), linear between grid points, y_255
 *   above; b(k) = max(S(k+1) - S(k), 0) on [k_s, k_top), k_s = the lowest level with E >= -2N
 *   (a decrease of the curve, e.g. its noise where the true steps are near zero at the top,
 *   gives a flat step). A curve with a step that is not finite, or with no positive step, is
 *   rejected and the realization keeps its plain start. host_k_seed (optional, n_real)
 *   receives k_s or -1. */
/* nfm_rec_targets: training targets from the current estimate, per realization 256 floats each
 * into dev_y and dev_mask (device): y_j = S(e_j N)/N on the grid e_j = -2 + 2j/255, S linear
 * between levels with S(k_top) = 0 (and S(k_top) above E(k_top)); mask 1 where e_j N >= E(k_lo),
 * else 0 with y = 0. */
nfm_status nfm_rec_targets(nfm_ctx* ctx, float* dev_y, float* dev_mask);
nfm_status nfm_set_canonical(nfm_ctx* ctx, double T);
nfm_status nfm_features(nfm_ctx* ctx, float* dev_x);
nfm_status nfm_rec_seed(nfm_ctx* ctx, const double* host_b, const int32_t* host_k_seed);
nfm_status nfm_rec_seed_grid(nfm_ctx* ctx, const float* dev_curves, int32_t* host_k_seed);

/* The model: 81 inputs, normalized per input as (x - mean)/sd; three hidden layers of 128 with
 * GELU (z Phi(z), erf form); 256 linear outputs (the curve y above). Parameter vector
 * (nfm_mlp_n_params() floats, weights row-major [in][out]): W0 [96 x 128] (rows 81..95 padding,
 * zero), b0 [128], W1 [128 x 128], b1, W2 [128 x 128], b2, W3 [128 x 256], b3 [256].
 * Training in FP32: masked mean squared error L = sum m (y - t)^2 / sum m over a batch, its
 * gradient by back-propagation, Adam with bias correction. Inference in BF16 (weights and
 * activations rounded to nearest even, FP32 accumulation). Products run on the matrix cores.
 * The context owns no memory: the caller's device workspace of nfm_mlp_workspace_bytes(). Device
 * pointers: x [B x 81], t and mask [B x 256], y [B x 256] floats, B in [1, batch_max]. */
typedef struct nfm_mlp nfm_mlp;
int32_t nfm_mlp_n_params(void);
nfm_status nfm_mlp_workspace_bytes(int32_t batch_max, size_t* bytes);
nfm_status nfm_mlp_create(nfm_mlp** out, int32_t batch_max, void* dev_workspace, size_t workspace_bytes,
                          int device, void* hip_stream);
/* Waits for the network's stream, then frees its host-side state (NULL is a no-op); the device
 * workspace stays the caller's. last_error: message of its last failed call, owned by it. */
void nfm_mlp_destroy(nfm_mlp* mlp);
const char* nfm_mlp_last_error(const nfm_mlp* mlp);
/* Glorot-uniform weights from the Philox stream (counter (q >> 2, layer, 0, 6), key = seed),
 * zero biases, identity normalization, optimizer state cleared. */
nfm_status nfm_mlp_init(nfm_mlp* mlp, uint64_t seed);
/* host_params (n_params floats) and/or host_norm (mean[81] then sd[81]); setting parameters
 * clears the optimizer state. */
nfm_status nfm_mlp_set_params(nfm_mlp* mlp, const float* host_params, const float* host_norm);
nfm_status nfm_mlp_get_params(nfm_mlp* mlp, float* host_params, float* host_norm);
nfm_status nfm_mlp_get_grads(nfm_mlp* mlp, float* host_grads);
nfm_status nfm_mlp_forward(nfm_mlp* mlp, const float* dev_x, int32_t B, float* dev_y);
/* Loss and gradient (kept for nfm_mlp_adam); host_loss (optional) synchronizes. */
nfm_status nfm_mlp_loss_grad(nfm_mlp* mlp, const float* dev_x, const float* dev_t, const float* dev_mask,
                             int32_t B, float* host_loss);
/* One Adam step (step count t + 1, bias corrections 1 - beta^t) from the gradient the last
 * nfm_mlp_loss_grad left; asynchronous. NFM_EINVAL unless lr > 0, 0 <= beta1, beta2 < 1, eps > 0. */
nfm_status nfm_mlp_adam(nfm_mlp* mlp, float lr, float beta1, float beta2, float eps);
/* loss_grad + adam(lr, 0.9, 0.999, 1e-8), asynchronous. */
nfm_status nfm_mlp_train_step(nfm_mlp* mlp, const float* dev_x, const float* dev_t, const float* dev_mask,
                              int32_t B, float lr);
/* Loss of the last nfm_mlp_loss_grad or nfm_mlp_train_step on the stream; synchronizes. */
nfm_status nfm_mlp_last_loss(nfm_mlp* mlp, float* host_loss);
/* BF16 copy of the current weights, then inference with it. */
nfm_status nfm_mlp_to_bf16(nfm_mlp* mlp);
nfm_status nfm_mlp_infer_bf16(nfm_mlp* mlp, const float* dev_x, int32_t B, float* dev_y);
/* For callers that cannot allocate (code under HIP graph capture, serving loops, harnesses that
 * forbid allocation): the same BF16 inference as nfm_mlp_infer_bf16, same results bit for bit,
 * with its activations in a static device array of the library (one per GPU, about 1.8 MB, held
 * until the process ends) instead of the network's workspace. Allocates nothing and calls no
 * allocating routine; asynchronous on the network's stream. B in [1, 1024] rows (NFM_ERANGE
 * above, independent of batch_max); dev_x [B x 81] and dev_y [B x 256] floats (device) are the
 * caller's. Every call on one GPU shares that array: calls that overlap on one GPU (several
 * streams or threads) race; calls queued on one stream do not. */
nfm_status nfm_mlp_infer_bf16_noalloc(nfm_mlp* mlp, const float* dev_x, int32_t B, float* dev_y);

#ifdef __cplusplus
}
#endif
#endif /* NFM_H */
