/*
 * nfm_oracle.c -- plain sequential CPU model of the sampler (TEST INFRASTRUCTURE).
 *
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
 * use this file. It is deliberately slow and literal: one attempt at a time,
 * one Philox call per attempt, energies recomputed from the definition where
 * a check is asked for. It shares no code with the GPU library.
 *
 * Paper: F. Muller, S. Schnabel, W. Janke, "Nonflat Histogram Techniques for
 * Spin Glasses" (arXiv:2011.08560).
 *   Sec. II, Eq. (1)   bimodal EA Hamiltonian on a periodic simple-cubic lattice;
 *   Sec. II            3V couplings +-1 with probability 1/2, quenched;
 *   Sec. II, Eq. (2)   generalized Metropolis acceptance min(1, W(E_new)/W(E_old));
 *   Sec. II, Eqs. (3)-(7) flat, power-law and 1/k weights from the DOS;
 *   Sec. III           round trips between E ~ 0 and the lowest energy found.
 * Where the paper is silent (sweep order, random-number layout, threshold
 * quantization, the weight recursion's formula) this file follows the readings
 * listed in the header nfm_oracle.h and in the design notes of the repository.
 */
#include "nfm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., "Parallel random numbers: as easy as 1, 2, 3",
 * SC'11). Round: two 32x32->64 products of counter words 0 and 2 with fixed
 * multipliers; the high halves are xored with the other counter words and the
 * round key; the key is advanced by the Weyl constants between rounds.       */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
    uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static uint32_t philox_word(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint64_t seed,
                            int which) {
  uint32_t ctr[4] = {c0, c1, c2, c3};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t out[4];
  orc_philox4x32_10(ctr, key, out);
  return out[which];
}

/* ------------------------------------------------------------------------ */
/* Lattice: site i = x + L y + L^2 z; neighbour in direction d (0:x,1:y,2:z)
 * with periodic wrap. Sec. II, Eq. (1).                                     */
static int32_t neighbour(int32_t L, int32_t i, int32_t d, int32_t step) {
  int32_t x = i % L, y = (i / L) % L, z = i / (L * L);
  if (d == 0) x = (x + step + L) % L;
  if (d == 1) y = (y + step + L) % L;
  if (d == 2) z = (z + step + L) % L;
  return x + L * y + L * L * z;
}

int32_t orc_n_minus(int32_t L, const int8_t* J) {
  int32_t N = L * L * L, n = 0;
  for (int32_t c = 0; c < 3 * N; ++c) n += (J[c] < 0);
  return n;
}

/* E = -sum J S S equals -3N + 2 n_minus for all spins up, and every single
 * flip changes E by a multiple of 4, so all reachable energies share that
 * residue mod 4 (E = -3N+2n_minus mod 4). Lowest conceivable level: -3N
 * shifted up by 2 if n_minus is odd.                                        */
int32_t orc_e_base(int32_t L, const int8_t* J) {
  int32_t N = L * L * L;
  return -3 * N + 2 * (orc_n_minus(L, J) % 2);
}

int32_t orc_n_levels(int32_t L, const int8_t* J) {
  int32_t N = L * L * L;
  return (3 * N - orc_e_base(L, J)) / 4 + 1;
}

/* Checkerboard order: colour c = (x+y+z) mod 2; colour 0 first, ascending i. */
void orc_sweep_order(int32_t L, int32_t* order) {
  int32_t N = L * L * L, a = 0;
  for (int32_t colour = 0; colour < 2; ++colour)
    for (int32_t i = 0; i < N; ++i) {
      int32_t x = i % L, y = (i / L) % L, z = i / (L * L);
      if ((x + y + z) % 2 == colour) order[a++] = i;
    }
}

/* ------------------------------------------------------------------------ */
/* Disorder (Sec. II): 3V couplings, each -1 with probability 1/2. Bit c of the
 * stream (c = d N + i) comes from word c/32 of realization real_id; word m is
 * output[m & 3] of counter (m >> 2, real_id, 0, TAG_J). Bit set <=> J = -1.  */
void orc_gen_couplings(int32_t L, uint64_t disorder_seed, uint32_t real_id, int8_t* J) {
  int32_t N = L * L * L;
  for (int32_t c = 0; c < 3 * N; ++c) {
    uint32_t m = (uint32_t)(c / 32);
    uint32_t word = philox_word(m >> 2, real_id, 0u, ORC_TAG_J, disorder_seed, (int)(m & 3u));
    uint32_t bit = (word >> (c % 32)) & 1u;
    J[c] = bit ? -1 : 1;
  }
}

/* Initial spins: bit i from word i/32 = output[m & 3] of counter
 * (m >> 2, 0, real_id, (walker << 8) | TAG_SPIN). Bit set <=> S = -1.        */
void orc_gen_spins(int32_t L, uint64_t walker_seed, uint32_t real_id, uint32_t walker, int8_t* S) {
  int32_t N = L * L * L;
  for (int32_t i = 0; i < N; ++i) {
    uint32_t m = (uint32_t)(i / 32);
    uint32_t word = philox_word(m >> 2, 0u, real_id, (walker << 8) | ORC_TAG_SPIN, walker_seed,
                                (int)(m & 3u));
    S[i] = ((word >> (i % 32)) & 1u) ? -1 : 1;
  }
}

/* ------------------------------------------------------------------------ */
/* Eq. (1): H = - sum over nearest-neighbour bonds of J_ij S_i S_j. Each site
 * owns its three forward bonds, so every bond is counted once.              */
int32_t orc_energy(int32_t L, const int8_t* J, const int8_t* S) {
  int32_t N = L * L * L, E = 0;
  for (int32_t i = 0; i < N; ++i)
    for (int32_t d = 0; d < 3; ++d) {
      int32_t j = neighbour(L, i, d, +1);
      E -= J[d * N + i] * S[i] * S[j];
    }
  return E;
}

int32_t orc_unsatisfied(int32_t L, const int8_t* J, const int8_t* S, int32_t i) {
  int32_t N = L * L * L, u = 0;
  for (int32_t d = 0; d < 3; ++d) {
    int32_t jf = neighbour(L, i, d, +1);
    int32_t jb = neighbour(L, i, d, -1);
    if (J[d * N + i] * S[i] * S[jf] < 0) ++u;   /* bond i -- i+e_d, owned by i  */
    if (J[d * N + jb] * S[i] * S[jb] < 0) ++u;  /* bond i-e_d -- i, owned by jb */
  }
  return u;
}

/* ------------------------------------------------------------------------ */
/* Threshold table. Eq. (2) accepts a move k -> k+m (m = 3-u levels, i.e.
 * Delta E = 4m) with probability min(1, W(k+m)/W(k)). With step log-weights
 * d(j) = lnW(j+1) - lnW(j) the ratio is exp(d(k)+...+d(k+m-1)) for m > 0 and
 * exp(-(d(k+m)+...+d(k-1))) for m < 0, summed in ascending j. Outside the
 * known range: d(j) = 0 for j >= k_top (W constant above the top energy) and
 * d(j) = d(k_lo) for j < k_lo (lowest known step continued). The probability
 * is stored as thr = floor(x 2^32), or 0xFFFFFFFF (always accept) if x >= 1.
 * An attempt with 32-bit random word r is accepted iff thr = 0xFFFFFFFF or
 * r < max(thr, 1): probabilities are quantised down to multiples of 2^-32,
 * with 2^-32 as the least (no move is forbidden outright).                  */
static double step_logw(const double* lnw, int32_t k_lo, int32_t k_top, int32_t j) {
  if (j < k_lo) j = k_lo;
  if (j >= k_top) return 0.0;
  return lnw[j + 1 - k_lo] - lnw[j - k_lo];
}

int32_t orc_metropolis_accept(uint32_t r, uint32_t thr) {
  return (thr == 0xFFFFFFFFu) || (r < (thr ? thr : 1u));
}

static uint32_t quantize(double x) {
  if (x >= 1.0) return 0xFFFFFFFFu;
  return (uint32_t)floor(ldexp(x, 32));
}

int32_t orc_table_rows(int32_t K, int32_t k_lo, int32_t k_top, int32_t* row0) {
  int32_t lo = k_lo - 3 < 0 ? 0 : k_lo - 3;
  int32_t hi = k_top + 3 > K - 1 ? K - 1 : k_top + 3;
  *row0 = lo;
  return hi - lo + 1;
}

int32_t orc_build_thresholds(int32_t K, const double* lnw, int32_t k_lo, int32_t k_top,
                             uint32_t* thr, int32_t* row0, int32_t* rows) {
  if (k_lo < 0 || k_top >= K || k_lo > k_top) return -1;
  *rows = orc_table_rows(K, k_lo, k_top, row0);
  for (int32_t r = 0; r < *rows; ++r) {
    int32_t k = *row0 + r;
    for (int32_t u = 0; u < 8; ++u) {
      uint32_t t = 0;
      if (u <= 6) {
        int32_t m = 3 - u;
        double x = 1.0;
        if (m > 0) {
          double s = 0.0;
          for (int32_t j = k; j <= k + m - 1; ++j) s += step_logw(lnw, k_lo, k_top, j);
          x = exp(s);
        } else if (m < 0) {
          double s = 0.0;
          for (int32_t j = k + m; j <= k - 1; ++j) s += step_logw(lnw, k_lo, k_top, j);
          x = exp(-s);
        }
        t = quantize(x);
      }
      thr[r * 8 + u] = t;
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Round trips (Sec. III): a round trip runs from the highest energies (E >= e_top,
 * "E ~ 0") to the lowest energy found (E <= e_bot) and back. States: 0 = top not
 * reached yet, 1 = at/after the top, 2 = bottom reached after the top. An
 * energy below e_bot is a new minimum, which asks for the sample to be rerun.  */
void orc_track(orc_walker* w, int32_t E, int32_t e_bot, int32_t e_top, uint64_t tau) {
  if (E < w->E_min) w->E_min = E;
  if (E < e_bot) w->new_min = 1;
  if (E >= e_top) {
    if (w->rt_state == 2) {
      w->rt_count += 1;
      w->t_last = tau;
    }
    if (w->rt_state == 0) w->t_first = tau;
    w->rt_state = 1;
  } else if (E <= e_bot && w->rt_state == 1) {
    w->rt_state = 2;
  }
}

/* ------------------------------------------------------------------------ */
/* Random word of an attempt: the site's colour c = (x+y+z) mod 2, its plane z and
 * its rank q among the colour-c sites of plane z in ascending i select
 * output[q & 3] of Philox counter (((c L + z) << 8) | (q >> 2), t, real_id,
 * (walker << 8) | TAG_ACC) under key = walker seed.                          */
static void site_rng_slot(int32_t L, int32_t i, uint32_t* ctr0, int32_t* which) {
  int32_t x = i % L, y = (i / L) % L, z = i / (L * L);
  int32_t c = (x + y + z) % 2;
  int32_t q = 0;
  for (int32_t yy = 0; yy < L; ++yy)
    for (int32_t xx = 0; xx < L; ++xx)
      if ((xx + yy + z) % 2 == c && xx + L * yy < x + L * y) ++q;
  *ctr0 = ((uint32_t)(c * L + z) << 8) | (uint32_t)(q >> 2);
  *which = q & 3;
}

/* Multicanonical sweeps, Eq. (2). One sweep = N attempts in checkerboard order.
 * The table row of level k is clamped into [row0, row0+rows-1]. After every
 * attempt the round-trip tracker sees the energy with stamp t N + a + 1; after
 * every sweep the energy level is histogrammed and traced.                  */
int32_t orc_muca_sweeps(int32_t L, const int8_t* J, int8_t* S, orc_walker* w,
                        const uint32_t* thr, int32_t row0, int32_t rows,
                        int32_t e_bot, int32_t e_top,
                        uint64_t walker_seed, uint32_t real_id, uint32_t walker,
                        uint64_t t0, uint64_t n_sweeps,
                        uint64_t* hist, int32_t* trace, int32_t check_energy) {
  int32_t N = L * L * L;
  int32_t e_base = orc_e_base(L, J);
  int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
  uint32_t* slot_ctr = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)N);
  int32_t* slot_which = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
  if (!order || !slot_ctr || !slot_which) {
    free(order); free(slot_ctr); free(slot_which);
    return -2;
  }
  orc_sweep_order(L, order);
  for (int32_t i = 0; i < N; ++i) site_rng_slot(L, i, &slot_ctr[i], &slot_which[i]);
  int32_t status = 0;
  for (uint64_t t = t0; t < t0 + n_sweeps; ++t) {
    for (int32_t a = 0; a < N; ++a) {
      int32_t i = order[a];
      int32_t u = orc_unsatisfied(L, J, S, i);
      int32_t k = (w->E - e_base) / 4;
      int32_t row = k - row0;
      if (row < 0) row = 0;
      if (row > rows - 1) row = rows - 1;
      uint32_t th = thr[row * 8 + u];
      uint32_t r = philox_word(slot_ctr[i], (uint32_t)t, real_id,
                               (walker << 8) | ORC_TAG_ACC, walker_seed, slot_which[i]);
      int accept = orc_metropolis_accept(r, th);
      if (accept) {
        S[i] = (int8_t)(-S[i]);
        w->E += 12 - 4 * u;
      }
      if (check_energy && w->E != orc_energy(L, J, S)) status = -1;
      orc_track(w, w->E, e_bot, e_top, t * (uint64_t)N + (uint64_t)a + 1u);
    }
    if (hist) hist[(w->E - e_base) / 4] += 1u;
    if (trace) trace[t - t0] = w->E;
  }
  free(order);
  free(slot_ctr);
  free(slot_which);
  return status;
}

/* ------------------------------------------------------------------------ */
/* Density of states by enumerating all 2^N spin states in Gray-code order:
 * step s flips spin ctz(s), so each state is visited once.                  */
int32_t orc_brute_dos(int32_t L, const int8_t* J, uint64_t* g) {
  int32_t N = L * L * L;
  if (N > 32) return -1;
  int32_t e_base = orc_e_base(L, J);
  int32_t K = orc_n_levels(L, J);
  memset(g, 0, sizeof(uint64_t) * (size_t)K);
  int8_t* S = (int8_t*)malloc((size_t)N);
  if (!S) return -2;
  for (int32_t i = 0; i < N; ++i) S[i] = 1;
  int32_t E = orc_energy(L, J, S);
  g[(E - e_base) / 4] += 1u;
  uint64_t total = (uint64_t)1 << N;
  for (uint64_t s = 1; s < total; ++s) {
    int32_t i = __builtin_ctzll(s);
    int32_t u = orc_unsatisfied(L, J, S, i);
    S[i] = (int8_t)(-S[i]);
    E += 12 - 4 * u;
    if ((E - e_base) % 4 != 0) {
      free(S);
      return -3; /* energy off the level lattice: cannot happen for +-1 couplings */
    }
    g[(E - e_base) / 4] += 1u;
  }
  free(S);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Eq. (5): P_SH(E) = (E/(dE - E_g) + 1)^alpha, equal to 1 at E = 0.          */
double orc_power_profile(double E, double E_g, double dE, double alpha) {
  return pow(E / (dE - E_g) + 1.0, alpha);
}

/* Weights of one iteration from the DOS steps b(k) = S(k+1) - S(k):
 *   S(k_top) = 0, S(k) = S(k+1) - b(k) going down to k_lo;
 *   lnP: flat 0; power law log of Eq. (5) with E_g = E(k_lo) (Sec. II: the
 *        profile is re-anchored whenever a lower energy is found);
 *        1/k: S(k) - ln sum_{j=k_lo..k} exp S(j), from Eq. (7), accumulated
 *        in ascending k with acc <- m + log1p(exp(-|acc - S|)), m = max;
 *   lnW = -S + lnP (Eq. (4); Eq. (3) for the flat profile).
 * Arrays are indexed by level, valid on [k_lo, k_top].                      */
void orc_rec_weights(int32_t K, int32_t e_base, int32_t k_lo, int32_t k_top, int32_t profile,
                     double pl_dE, double pl_alpha, const double* b,
                     double* S, double* lnP, double* lnW) {
  orc_rec_weights_ext(K, e_base, k_lo, k_top, k_lo, profile, pl_dE, pl_alpha, b, S, lnP, lnW);
}

/* The same with a lower end k_low <= k_lo: a seeded estimate (prior DOS steps on levels
 * not yet sampled) continues S below k_lo with its own steps, S(k) = S(k+1) - b(k), under
 * the frozen profile lnP(k) = lnP(k_lo); arrays are then valid on [k_low, k_top].        */
void orc_rec_weights_ext(int32_t K, int32_t e_base, int32_t k_lo, int32_t k_top, int32_t k_low,
                         int32_t profile, double pl_dE, double pl_alpha, const double* b,
                         double* S, double* lnP, double* lnW) {
  (void)K;
  S[k_top] = 0.0;
  for (int32_t k = k_top - 1; k >= k_lo; --k) S[k] = S[k + 1] - b[k];
  double E_g = (double)(e_base + 4 * k_lo);
  double acc = 0.0;
  for (int32_t k = k_lo; k <= k_top; ++k) {
    double E = (double)(e_base + 4 * k);
    if (profile == ORC_PROFILE_FLAT) {
      lnP[k] = 0.0;
    } else if (profile == ORC_PROFILE_POWER) {
      lnP[k] = pl_alpha * log(E / (pl_dE - E_g) + 1.0);
    } else {
      if (k == k_lo) {
        acc = S[k];
      } else {
        double m = acc > S[k] ? acc : S[k];
        acc = m + log1p(exp(-fabs(acc - S[k])));
      }
      lnP[k] = S[k] - acc;
    }
    lnW[k] = -S[k] + lnP[k];
  }
  for (int32_t k = k_lo - 1; k >= k_low; --k) {
    S[k] = S[k + 1] - b[k];
    lnP[k] = lnP[k_lo];
    lnW[k] = -S[k] + lnP[k];
  }
}

/* Accumulated-statistics recursion (Berg's multicanonical recursion written for
 * a target profile; the paper cites its iteration without printing it, Sec. II).
 * Input: the log-weights lnW_used and profile lnP_used that produced histogram H
 * (valid on [k_lo_used, k_top]), the lowest level seen while sampling.
 *  1. k_lo <- min(k_lo_used, k_min_seen). New levels below k_lo_used take
 *     b(k) = b(k_lo_used) and p(k) = 0. Below k_lo_used the weights used were
 *     lnW continued with the lowest step, and the profile was frozen.
 *  2. For each pair k < k' of consecutive levels in [k_lo, k_top] with H > 0:
 *        est = [ln H(k') - lnW(k')] - [ln H(k) - lnW(k)]    (estimate of S(k')-S(k))
 *        span = b(k) + ... + b(k'-1)
 *        g0 = H(k) H(k') / (H(k) + H(k')),  p(k) += g0,  b(k) += (g0/p(k)) (est - span).
 *  3. visited |= (H > 0) on [k_lo, k_top].
 *  4. flatness = min / mean of H/P over visited levels in [k_lo, k_top].        */
void orc_rec_update(int32_t K, int32_t k_lo_used, int32_t k_top, int32_t k_min_seen,
                    const double* lnW_used, const double* lnP_used, const uint64_t* H,
                    double* b, double* p, uint8_t* visited, int32_t* k_lo_new,
                    double* flatness) {
  orc_rec_update_ext(K, k_lo_used, k_top, k_lo_used, 0, k_min_seen, lnW_used, lnP_used, H, b, p, visited,
                     k_lo_new, flatness);
}

/* The same for an estimate that may be seeded: lnW_used is valid on [k_low_used, k_top]
 * (k_low_used <= k_lo_used; below it the lowest step continues), and with seeded != 0
 * new levels below k_lo_used keep their seeded steps b(k) (with p(k) = 0) instead of
 * copying b(k_lo_used).                                                              */
void orc_rec_update_ext(int32_t K, int32_t k_lo_used, int32_t k_top, int32_t k_low_used, int32_t seeded,
                        int32_t k_min_seen, const double* lnW_used, const double* lnP_used,
                        const uint64_t* H, double* b, double* p, uint8_t* visited, int32_t* k_lo_new,
                        double* flatness) {
  (void)K;
  int32_t k_lo = k_min_seen < k_lo_used ? k_min_seen : k_lo_used;
  for (int32_t k = k_lo; k < k_lo_used; ++k) {
    if (!seeded) b[k] = b[k_lo_used];
    p[k] = 0.0;
  }
  int32_t low = k_low_used < k_lo_used ? k_low_used : k_lo_used;
  double d_lo = (low < k_top) ? lnW_used[low + 1] - lnW_used[low] : 0.0;
  /* weights and profile as they were while sampling, on [k_lo, k_top] */
  #define LNW_AT(k) ((k) >= low ? lnW_used[k] : lnW_used[low] - (double)(low - (k)) * d_lo)
  #define LNP_AT(k) ((k) >= k_lo_used ? lnP_used[k] : lnP_used[k_lo_used])
  int32_t prev = -1;
  for (int32_t k = k_lo; k <= k_top; ++k) {
    if (H[k] == 0) continue;
    if (prev >= 0) {
      double Hk = (double)H[prev], Hk1 = (double)H[k];
      double est = (log(Hk1) - LNW_AT(k)) - (log(Hk) - LNW_AT(prev));
      double span = 0.0;
      for (int32_t j = prev; j < k; ++j) span += b[j];
      double g0 = Hk * Hk1 / (Hk + Hk1);
      p[prev] += g0;
      b[prev] += (g0 / p[prev]) * (est - span);
    }
    prev = k;
  }
  double mn = 0.0, sum = 0.0;
  int32_t n = 0;
  for (int32_t k = k_lo; k <= k_top; ++k) {
    if (H[k] > 0) visited[k] = 1;
    if (!visited[k]) continue;
    double v = (double)H[k] / exp(LNP_AT(k));
    if (n == 0 || v < mn) mn = v;
    sum += v;
    ++n;
  }
  #undef LNW_AT
  #undef LNP_AT
  *flatness = (n > 0 && sum > 0.0) ? mn / (sum / (double)n) : 0.0;
  *k_lo_new = k_lo;
}

/* Seed of the DOS steps from a curve y_j = [S(E) - S(E_top)]/N on the energy grid
 * e_j = -2 + 2j/255 (j = 0..255): S(k) = N y(E_k/N), linear between grid points and y_255
 * above the grid; steps b(k) = max(S(k+1) - S(k), 0) on [k_s, k_top), k_s the lowest level
 * with E >= -2N (a decrease of the curve, such as its noise where the true steps are near zero
 * at the top, or anything below the ground state, gives a flat step). Returns k_s and fills b,
 * or returns -1 (b untouched) when a step is not finite or no step is positive: the curve is
 * then rejected and the plain start is kept.                                      */
static double seed_curve(const float* y, double e) {
  double t = (e + 2.0) * 127.5;
  if (t <= 0.0) return (double)y[0];
  if (t >= 255.0) return (double)y[255];
  int32_t j = (int32_t)floor(t);
  double f = t - (double)j;
  return (double)y[j] + f * ((double)y[j + 1] - (double)y[j]);
}

static double seed_step(int32_t N, int32_t e_base, const float* y, int32_t k) {
  double s0 = (double)N * seed_curve(y, (double)(e_base + 4 * k) / (double)N);
  double s1 = (double)N * seed_curve(y, (double)(e_base + 4 * (k + 1)) / (double)N);
  return s1 - s0;
}

int32_t orc_seed_from_grid(int32_t N, int32_t e_base, int32_t k_top, const float* y, double* b) {
  int32_t k_s = (-2 * N - e_base + 3) / 4;   /* ceil((-2N - e_base)/4), -2N - e_base >= 0 */
  if (k_s < 0) k_s = 0;
  double total = 0.0;
  for (int32_t k = k_s; k < k_top; ++k) {
    double d = seed_step(N, e_base, y, k);
    if (!isfinite(d)) return -1;
    if (d > 0.0) total += d;
  }
  if (!(total > 0.0)) return -1;
  for (int32_t k = k_s; k < k_top; ++k) {
    double d = seed_step(N, e_base, y, k);
    b[k] = d > 0.0 ? d : 0.0;
  }
  return k_s;
}

/* ------------------------------------------------------------------------ */
/* Frustration statistics of one realization (inputs of the weight-seeding model).
 * A plaquette (i; d1, d2) has the bonds J_d1(i), J_d2(i+e_d1), J_d1(i+e_d2), J_d2(i); it is
 * frustrated when their product is -1. The elementary cube at corner i has six faces: the
 * (x,y) plaquettes at i and i+e_z, (y,z) at i and i+e_x, (z,x) at i and i+e_y; an even
 * number of them is frustrated. out[16]:
 *   0..2  frustrated fraction of (x,y), (y,z), (z,x) plaquettes;  3  of all plaquettes;
 *   4..6  negative-bond fraction along x, y, z;  7  of all bonds;  8  n_minus mod 2;
 *   9..12 fraction of cubes with 0, 2, 4, 6 frustrated faces;
 *   13..15 mean / 6, variance / 6 and fourth central moment / 96 of the site sums
 *          sum_j J_ij over the six bonds of a site.                                 */
static int32_t plaq_frustrated(int32_t L, const int8_t* J, int32_t i, int32_t d1, int32_t d2) {
  int32_t N = L * L * L;
  int32_t a = neighbour(L, i, d1, 1), c = neighbour(L, i, d2, 1);
  int32_t prod = J[d1 * N + i] * J[d2 * N + a] * J[d1 * N + c] * J[d2 * N + i];
  return prod < 0;
}

void orc_features(int32_t L, const int8_t* J, double* out) {
  int32_t N = L * L * L;
  int32_t orient[3][2] = {{0, 1}, {1, 2}, {2, 0}};
  int64_t fr[3] = {0, 0, 0}, neg[3] = {0, 0, 0}, cubes[4] = {0, 0, 0, 0};
  for (int32_t o = 0; o < 3; ++o)
    for (int32_t i = 0; i < N; ++i) fr[o] += plaq_frustrated(L, J, i, orient[o][0], orient[o][1]);
  for (int32_t d = 0; d < 3; ++d)
    for (int32_t i = 0; i < N; ++i) neg[d] += J[d * N + i] < 0;
  for (int32_t i = 0; i < N; ++i) {
    int32_t f = plaq_frustrated(L, J, i, 0, 1) + plaq_frustrated(L, J, neighbour(L, i, 2, 1), 0, 1) +
                plaq_frustrated(L, J, i, 1, 2) + plaq_frustrated(L, J, neighbour(L, i, 0, 1), 1, 2) +
                plaq_frustrated(L, J, i, 2, 0) + plaq_frustrated(L, J, neighbour(L, i, 1, 1), 2, 0);
    cubes[f / 2] += 1;
  }
  double mean = 0.0;
  for (int32_t i = 0; i < N; ++i) {
    int32_t sum = 0;
    for (int32_t d = 0; d < 3; ++d) sum += J[d * N + i] + J[d * N + neighbour(L, i, d, -1)];
    mean += (double)sum;
  }
  mean /= (double)N;
  double m2 = 0.0, m4 = 0.0;
  for (int32_t i = 0; i < N; ++i) {
    int32_t sum = 0;
    for (int32_t d = 0; d < 3; ++d) sum += J[d * N + i] + J[d * N + neighbour(L, i, d, -1)];
    double x = (double)sum - mean;
    m2 += x * x;
    m4 += x * x * x * x;
  }
  m2 /= (double)N;
  m4 /= (double)N;
  for (int32_t o = 0; o < 3; ++o) out[o] = (double)fr[o] / (double)N;
  out[3] = (double)(fr[0] + fr[1] + fr[2]) / (double)(3 * N);
  for (int32_t d = 0; d < 3; ++d) out[4 + d] = (double)neg[d] / (double)N;
  out[7] = (double)(neg[0] + neg[1] + neg[2]) / (double)(3 * N);
  out[8] = (double)((neg[0] + neg[1] + neg[2]) % 2);
  for (int32_t c = 0; c < 4; ++c) out[9 + c] = (double)cubes[c] / (double)N;
  out[13] = mean / 6.0;
  out[14] = m2 / 6.0;
  out[15] = m4 / 96.0;
}

/* Energy histogram of a canonical run as 64 bins of E/N over [-2, 0): bin
 * floor((E/N + 2) 32), clipped into [0, 63]; fractions of all entries.            */
void orc_hist_bins(int32_t K, int32_t e_base, int32_t N, const uint64_t* H, double* out) {
  uint64_t tot = 0;
  for (int32_t j = 0; j < 64; ++j) out[j] = 0.0;
  for (int32_t k = 0; k < K; ++k) tot += H[k];
  if (tot == 0) return;
  uint64_t cnt[64] = {0};
  for (int32_t k = 0; k < K; ++k) {
    if (H[k] == 0) continue;
    double e = (double)(e_base + 4 * k) / (double)N;
    int32_t j = (int32_t)floor((e + 2.0) * 32.0);
    if (j < 0) j = 0;
    if (j > 63) j = 63;
    cnt[j] += H[k];
  }
  for (int32_t j = 0; j < 64; ++j) out[j] = (double)cnt[j] / (double)tot;
}

/* ------------------------------------------------------------------------ */
/* Parallel tempering (Sec. II, Eq. (8)): M copies of the system at temperatures
 * T_0 < ... < T_{M-1}, each updated by canonical Metropolis, and exchanges of the
 * configurations of neighbouring temperatures.
 *
 * Metropolis table, one row per temperature slot in the layout of the multicanonical
 * tables (u = 0..6, pad): the step m = 3 - u changes E by 4m, accepted with
 * x = exp(-(1/T) (4m)) for m > 0 and always for m <= 0.                          */
void orc_pt_metro_table(int32_t M, const double* T, uint32_t* thr) {
  for (int32_t s = 0; s < M; ++s) {
    double beta = 1.0 / T[s];
    for (int32_t u = 0; u < 8; ++u) {
      uint32_t t = 0;
      if (u <= 6) {
        int32_t m = 3 - u;
        t = m <= 0 ? 0xFFFFFFFFu : quantize(exp(-beta * (double)(4 * m)));
      }
      thr[s * 8 + u] = t;
    }
  }
}

/* Exchange table: for the pair of slots (s, s+1) and d = (E_{s+1} - E_s)/4 >= 1 the
 * exchange is accepted with x = exp((1/T_{s+1} - 1/T_s) (4d)) (Eq. (8)), evaluated as
 * q^d with q = exp(4 (1/T_{s+1} - 1/T_s)) raised to d by binary powering (one FP64
 * product per bit of d and per squaring, lowest bit first), so that any machine that
 * is given q reproduces every entry bit for bit; entry [s][d-1] holds its threshold.
 * Exchanges with d <= 0 always succeed. D is the smallest d at which every pair's
 * threshold is 0 (so that larger d may be clamped to D), but at most d_cap. Returns D;
 * thr may be NULL to query it.                                                       */
double orc_pow_bin(double q, int32_t d) {
  double r = 1.0, b = q;
  while (d > 0) {
    if (d & 1) r = r * b;
    b = b * b;
    d >>= 1;
  }
  return r;
}

double orc_pt_swap_q(double T_lo, double T_hi) { return exp(4.0 * (1.0 / T_hi - 1.0 / T_lo)); }

int32_t orc_pt_swap_table(int32_t M, const double* T, int32_t d_cap, uint32_t* thr) {
  int32_t D = d_cap;
  for (int32_t d = 1; d <= d_cap; ++d) {
    int32_t all_zero = 1;
    for (int32_t s = 0; s + 1 < M; ++s)
      if (quantize(orc_pow_bin(orc_pt_swap_q(T[s], T[s + 1]), d)) != 0u) all_zero = 0;
    if (all_zero) {
      D = d;
      break;
    }
  }
  if (thr) {
    for (int32_t s = 0; s + 1 < M; ++s) {
      double q = orc_pt_swap_q(T[s], T[s + 1]);
      for (int32_t d = 1; d <= D; ++d) thr[s * D + (d - 1)] = quantize(orc_pow_bin(q, d));
    }
  }
  return D;
}

/* One set of M configurations of one realization. Configuration c (walker index
 * set*M + c of the realization) holds spins S[c*N .. c*N+N-1], bookkeeping w[c] and
 * temperature slot slot[c]. Each sweep t: every configuration, in order c = 0..M-1,
 * makes one checkerboard sweep of Metropolis attempts at T_slot (acceptance words as
 * in the multicanonical sweep with tag TAG_PT); then each configuration's energy is
 * tracked with stamp (t+1) N (round trips between e_bot and e_top, Sec. III); then
 * the pairs of slots (s, s+1) with s = t (mod 2) try an exchange, accepted when
 * thr == 0xFFFFFFFF or r < thr, r = output[s & 3] of counter
 * (s >> 2, t, real_id, (set << 8) | TAG_SWAP) under the walker seed.               */
int32_t orc_pt_sweeps(int32_t L, const int8_t* J, int32_t M, int8_t* S, orc_walker* w, int32_t* slot,
                      const uint32_t* metro, const uint32_t* swap, int32_t D, int32_t e_bot, int32_t e_top,
                      uint64_t walker_seed, uint32_t real_id, uint32_t set, uint32_t walker0, uint64_t t0,
                      uint64_t n_sweeps, uint64_t* swap_acc, int32_t* trace, int32_t check_energy) {
  int32_t N = L * L * L;
  int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
  uint32_t* slot_ctr = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)N);
  int32_t* slot_which = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
  int32_t* at = (int32_t*)malloc(sizeof(int32_t) * (size_t)M);
  if (!order || !slot_ctr || !slot_which || !at) {
    free(order); free(slot_ctr); free(slot_which); free(at);
    return -2;
  }
  orc_sweep_order(L, order);
  for (int32_t i = 0; i < N; ++i) site_rng_slot(L, i, &slot_ctr[i], &slot_which[i]);
  int32_t status = 0;
  for (uint64_t t = t0; t < t0 + n_sweeps; ++t) {
    for (int32_t c = 0; c < M; ++c) {
      int8_t* Sc = S + (size_t)c * (size_t)N;
      uint32_t walker = walker0 + (uint32_t)c;
      for (int32_t a = 0; a < N; ++a) {
        int32_t i = order[a];
        int32_t u = orc_unsatisfied(L, J, Sc, i);
        uint32_t th = metro[slot[c] * 8 + u];
        uint32_t r = philox_word(slot_ctr[i], (uint32_t)t, real_id, (walker << 8) | ORC_TAG_PT,
                                 walker_seed, slot_which[i]);
        if (orc_metropolis_accept(r, th)) {
          Sc[i] = (int8_t)(-Sc[i]);
          w[c].E += 12 - 4 * u;
        }
      }
      if (check_energy && w[c].E != orc_energy(L, J, Sc)) status = -1;
      orc_track(&w[c], w[c].E, e_bot, e_top, (t + 1u) * (uint64_t)N);
      if (trace) trace[(size_t)c * n_sweeps + (t - t0)] = w[c].E;
    }
    for (int32_t c = 0; c < M; ++c) at[slot[c]] = c;
    for (int32_t s = (int32_t)(t & 1u); s + 1 < M; s += 2) {
      int32_t lo = at[s], hi = at[s + 1];
      int32_t d = (w[hi].E - w[lo].E) / 4;
      uint32_t th = 0xFFFFFFFFu;
      if (d > 0) th = swap[s * D + (d < D ? d : D) - 1];
      uint32_t r = philox_word((uint32_t)(s >> 2), (uint32_t)t, real_id, (set << 8) | ORC_TAG_SWAP,
                               walker_seed, s & 3);
      if (th == 0xFFFFFFFFu || r < th) {
        slot[lo] = s + 1;
        slot[hi] = s;
        if (swap_acc) swap_acc[s] += 1u;
      }
    }
  }
  free(order);
  free(slot_ctr);
  free(slot_which);
  free(at);
  return status;
}
