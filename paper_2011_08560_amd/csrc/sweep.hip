// Multicanonical Metropolis sweeps (Sec. II, Eq. (2)) with per-attempt minimum and
// round-trip bookkeeping (Sec. III) and per-sweep histograms.
//
// Mapping: one lane = one walker; one wave = 64 walkers of one realization, which
// share its couplings (wave-uniform, scalar registers) and its threshold table
// (LDS). A walker's lattice stays in VGPRs for the whole launch, bit-packed by
// colour and plane (see nfm_internal.hpp).
//
// The sweep order is checkerboard: all sites of colour 0, then colour 1. The
// neighbours of a site all have the other colour, so at the start of each
// (colour, plane) block the number u of unsatisfied bonds of every site of the
// block is fixed; it is computed for the whole block at once with word-parallel
// bit operations (six flag strings and a bit-sliced adder). The attempts then run
// one after the other, since each acceptance reads the walker's current energy.
//
// Kernel forms: k_sweeps (one wave per workgroup; compact or expanded table, speculative or
// plain, tempering), k_sweeps_ws (the sampling wave plus a generator wave that supplies its
// random words through LDS) and k_sweeps_queue (persistent, over a batch of mixed sizes). All
// forms draw the same words for the same attempts, so their results are identical.
#include <algorithm>
#include <cstdio>
#include <type_traits>

#include "kernels.hpp"
#include "philox.hpp"

namespace nfm {

template <int L>
struct Geo {
  static constexpr int F = field_bits(L);
  static constexpr int NWP = plane_words(L);
  static constexpr int H = L / 2;           // sites of one colour per row
  static constexpr int Q = L * L / 2;       // sites of one colour per plane
  static constexpr int N = L * L * L;
  static constexpr int BITS = L * F;
  using PW = typename std::conditional<(BITS <= 32), uint32_t, __uint128_t>::type;

  // bits [lo, lo+width) of every field
  static constexpr PW fields(int lo, int width) {
    PW m = 0;
    for (int y = 0; y < L; ++y)
      for (int b = lo; b < lo + width; ++b) m |= PW(1) << (y * F + b);
    return m;
  }
  // valid bits of the rows y with y % 2 == parity
  static constexpr PW rows_of_parity(int parity) {
    PW m = 0;
    for (int y = parity; y < L; y += 2)
      for (int b = 0; b < H; ++b) m |= PW(1) << (y * F + b);
    return m;
  }
  static constexpr PW all_bits() {
    PW m = 0;
    for (int b = 0; b < BITS; ++b) m |= PW(1) << b;
    return m;
  }
};

template <int L>
__device__ __forceinline__ typename Geo<L>::PW pack(const uint32_t* w) {
  using G = Geo<L>;
  typename G::PW v = 0;
#pragma unroll
  for (int i = 0; i < G::NWP; ++i) v |= typename G::PW(w[i]) << (32 * i);
  return v;
}

template <int L>
__device__ __forceinline__ void unpack(typename Geo<L>::PW v, uint32_t* w) {
  using G = Geo<L>;
#pragma unroll
  for (int i = 0; i < G::NWP; ++i) w[i] = (uint32_t)(v >> (32 * i));
}


__device__ __forceinline__ int floor_div4(int a) { return a >= 0 ? a / 4 : -((-a + 3) / 4); }
__device__ __forceinline__ int ceil_div4(int a) { return -floor_div4(-a); }

// Bookkeeping window of the round-trip state: while lo <= B <= hi an attempt cannot change it
// (B = (k - row0) * 32 for level k). The walker's minimum and new-minimum flag do not depend on the
// order of the attempts, so they are taken from each group's lowest B instead; only a group in
// which some walker reached the bound its state waits for is replayed in order.
struct Window {
  int lo, hi;
};

// Groups of four attempts between two window checks of an L x L x L lattice. Each check costs the
// extremes of the levels since the last one, a compare and a branch, and a replay covers every
// attempt since then: a lone wave on its SIMD (the largest lattices) gains from longer intervals,
// several waves per SIMD whose walkers often reach a bound (small lattices, first rounds) from
// shorter ones.
template <int L>
constexpr int check_groups() { return L >= 12 ? 8 : L >= 10 ? 4 : 2; }

__device__ __forceinline__ Window make_window(int state, int Bbot, int Btop) {
  constexpr int INF = 1 << 29;
  Window w;
  w.lo = (state == 1) ? Bbot + 32 : -INF;   // at or after the top: waiting for the bottom
  w.hi = (state == 1) ? INF : Btop - 32;    // before the first top, or after a bottom: for the top
  return w;
}

// Exact round-trip bookkeeping of one attempt (Sec. III): E >= e_top <=> B >= Btop and
// E <= e_bot <=> B <= Bbot.
struct Track {
  int Bmin, state, newmin;
  uint32_t trips;
  uint64_t t_first, t_last;
};

__device__ __forceinline__ void track_attempt(Track& tr, int B, uint64_t tau, int Bbot, int Btop) {
  if (B >= Btop) {
    if (tr.state == 2) {
      tr.trips += 1;
      tr.t_last = tau;
    }
    if (tr.state == 0) tr.t_first = tau;
    tr.state = 1;
  } else if (B <= Bbot && tr.state == 1) {
    tr.state = 2;
  }
}

// Round-trip bookkeeping on energies, applied once per sweep (parallel tempering: a
// configuration's energy is examined after each Metropolis phase).
struct TrackE {
  int Emin, state, newmin;
  uint32_t trips;
  uint64_t t_first, t_last;
};

__device__ __forceinline__ void track_energy(TrackE& tr, int E, uint64_t tau, int e_bot, int e_top) {
  if (E < tr.Emin) tr.Emin = E;
  if (E < e_bot) tr.newmin = 1;
  if (E >= e_top) {
    if (tr.state == 2) {
      tr.trips += 1;
      tr.t_last = tau;
    }
    if (tr.state == 0) tr.t_first = tau;
    tr.state = 1;
  } else if (E <= e_bot && tr.state == 1) {
    tr.state = 2;
  }
}

__device__ __forceinline__ int lds_load_i32(uint32_t byte_addr) {
  return *(const __attribute__((address_space(3))) int*)(uintptr_t)byte_addr;
}
__device__ __forceinline__ void lds_store_i32(uint32_t byte_addr, int v) {
  *(__attribute__((address_space(3))) int*)(uintptr_t)byte_addr = v;
}
typedef uint32_t lds_v4u __attribute__((ext_vector_type(4)));
__device__ __forceinline__ u32x4 lds_load_u32x4(uint32_t byte_addr) {
  const lds_v4u q = *(const __attribute__((address_space(3))) lds_v4u*)(uintptr_t)byte_addr;
  return u32x4{{q.x, q.y, q.z, q.w}};
}
__device__ __forceinline__ void lds_store_u32x4(uint32_t byte_addr, const u32x4& w) {
  const lds_v4u q = {w.v[0], w.v[1], w.v[2], w.v[3]};
  *(__attribute__((address_space(3))) lds_v4u*)(uintptr_t)byte_addr = q;
}

// Warp-specialized form (expanded table only): a workgroup of two waves, the sampling wave and
// a generator wave that computes the random words of the sampling wave's walkers two blocks
// ahead into a ring of three block slots in LDS (16 bytes per walker and group of four sites),
// after the sampling wave's table, couplings and histogram. Both waves meet at one barrier per
// block. The generator's work leaves the sampling wave's instruction stream, and the two waves
// share a SIMD's issue slots where one wave per SIMD would leave them idle.
template <int L>
__host__ __device__ constexpr uint32_t ws_slot_bytes() {
  return (uint32_t)((Geo<L>::Q + 3) / 4) * 64u * 16u;
}
__host__ __device__ inline uint32_t ws_ring_base(int K, int jk_words_L, int hist_n) {
  return ((uint32_t)K * 32u + 4u * (uint32_t)jk_words_L + 4u * (uint32_t)hist_n + 15u) & ~15u;
}

// Acceptance of one attempt and its effect on the state, as one instruction sequence: the
// comparison r <= th' of the random word with the on-chip threshold (th' = thr - 1, or 0 for
// thr = 0, or 2^32 - 1 for always, so that r <= th' <=> thr = 2^32 - 1 or r < max(thr, 1)) sets VCC, which then selects the new state and is shifted into the flip word F
// (F = 2F + accepted). The two instructions between the comparison and the first reader of
// VCC are the distance the hardware needs between a VALU write of VCC and a VALU read of it.
//   level form:  B (row offset of the level, 32 per level) += 32 m on acceptance
//   energy form: E += 4 m on acceptance (tempering: the row is the temperature slot)
// m = the sign-extended 3-bit field at bits 2..4 of hi.
// hn: the next site's gathered field; addr receives the next site's table address.
__device__ __forceinline__ void accept_level(uint32_t rc, uint32_t th, uint32_t hi, uint32_t hn, int vBmax, int& B,
                                             int& R, uint32_t& F, uint32_t& addr) {
  int m, Bacc, Bn, Rn;
  uint32_t Fn, an;
  asm volatile("v_cmp_le_u32_e32 vcc, %[rc], %[th]\n\t"
      "v_bfe_i32 %[m], %[hi], 2, 3\n\t"
      "v_lshl_add_u32 %[Bacc], %[m], 5, %[B]\n\t"
      "v_cndmask_b32_e32 %[Bn], %[B], %[Bacc], vcc\n\t"
      "v_addc_co_u32_e32 %[Fn], vcc, %[F], %[F], vcc\n\t"
      "v_med3_i32 %[Rn], %[Bn], 0, %[Bmax]\n\t"
      "v_and_or_b32 %[an], %[hn], 28, %[Rn]"
      : [Bn] "=&v"(Bn), [Rn] "=&v"(Rn), [Fn] "=&v"(Fn), [m] "=&v"(m), [Bacc] "=&v"(Bacc), [an] "=&v"(an)
      : [rc] "v"(rc), [th] "v"(th), [hi] "v"(hi), [hn] "v"(hn), [B] "v"(B), [F] "v"(F), [Bmax] "v"(vBmax)
      : "vcc");
  B = Bn;
  R = Rn;
  F = Fn;
  addr = an;
}

// Expanded table (every level has its own row on chip): the row is the level, no clamp.
__device__ __forceinline__ void accept_level_xt(uint32_t rc, uint32_t th, uint32_t hi, uint32_t hn, int& B,
                                                uint32_t& F, uint32_t& addr) {
  int m, Bacc, Bn;
  uint32_t Fn, an;
  asm volatile("v_cmp_le_u32_e32 vcc, %[rc], %[th]\n\t"
      "v_bfe_i32 %[m], %[hi], 2, 3\n\t"
      "v_lshl_add_u32 %[Bacc], %[m], 5, %[B]\n\t"
      "v_cndmask_b32_e32 %[Bn], %[B], %[Bacc], vcc\n\t"
      "v_addc_co_u32_e32 %[Fn], vcc, %[F], %[F], vcc\n\t"
      "v_and_or_b32 %[an], %[hn], 28, %[Bn]"
      : [Bn] "=&v"(Bn), [Fn] "=&v"(Fn), [m] "=&v"(m), [Bacc] "=&v"(Bacc), [an] "=&v"(an)
      : [rc] "v"(rc), [th] "v"(th), [hi] "v"(hi), [hn] "v"(hn), [B] "v"(B), [F] "v"(F)
      : "vcc");
  B = Bn;
  F = Fn;
  addr = an;
}

__device__ __forceinline__ void accept_energy(uint32_t rc, uint32_t th, uint32_t hi, int& E, uint32_t& F) {
  int m, Eacc, En;
  uint32_t Fn;
  asm volatile("v_cmp_le_u32_e32 vcc, %[rc], %[th]\n\t"
      "v_bfe_i32 %[m], %[hi], 2, 3\n\t"
      "v_lshl_add_u32 %[Eacc], %[m], 2, %[E]\n\t"
      "v_cndmask_b32_e32 %[En], %[E], %[Eacc], vcc\n\t"
      "v_addc_co_u32_e32 %[Fn], vcc, %[F], %[F], vcc"
      : [En] "=&v"(En), [Fn] "=&v"(Fn), [m] "=&v"(m), [Eacc] "=&v"(Eacc)
      : [rc] "v"(rc), [th] "v"(th), [hi] "v"(hi), [E] "v"(E), [F] "v"(F)
      : "vcc");
  E = En;
  F = Fn;
}

// Speculative form: the level and the clamped row after acceptance are computed beforehand
// (the next site's thresholds for both outcomes are loaded meanwhile).
__device__ __forceinline__ void accept_level_spec(uint32_t rc, uint32_t th, int Bacc, int Racc, int& B, int& R,
                                                  uint32_t& F) {
  int Bn, Rn;
  uint32_t Fn;
  asm("v_cmp_le_u32_e32 vcc, %[rc], %[th]\n\t"
      "s_nop 1\n\t"
      "v_cndmask_b32_e32 %[Bn], %[B], %[Bacc], vcc\n\t"
      "v_cndmask_b32_e32 %[Rn], %[R], %[Racc], vcc\n\t"
      "v_addc_co_u32_e32 %[Fn], vcc, %[F], %[F], vcc"
      : [Bn] "=&v"(Bn), [Rn] "=&v"(Rn), [Fn] "=&v"(Fn)
      : [rc] "v"(rc), [th] "v"(th), [Bacc] "v"(Bacc), [Racc] "v"(Racc), [B] "v"(B), [R] "v"(R), [F] "v"(F)
      : "vcc");
  B = Bn;
  R = Rn;
  F = Fn;
}

// Exchange threshold of slots (s, s+1) whose energies differ by 4d (Eq. (8)): q^d rounded down
// to a multiple of 2^-32 (0xFFFFFFFF = always, d <= 0), q = exp(4 (beta_{s+1} - beta_s)) given by
// the host, raised to d by binary powering (one FP64 product per bit and per squaring, lowest bit
// first) -- products only, so the host reproduces every value bit for bit.
__device__ __forceinline__ uint32_t pt_swap_threshold(double q, int d) {
  if (d <= 0) return 0xFFFFFFFFu;
  double r = 1.0, b = q;
  while (d > 0) {
    if (d & 1) r = r * b;
    b = b * b;
    d >>= 1;
  }
  return r >= 1.0 ? 0xFFFFFFFFu : (uint32_t)floor(ldexp(r, 32));
}

__device__ __forceinline__ int clamp_row(int B, int Bmax) {
  int R;
  asm("v_med3_i32 %0, %1, 0, %2" : "=v"(R) : "v"(B), "s"(Bmax));
  return R;
}

// PT = false: multicanonical sweeps; the table row follows the walker's level.
// PT = true: parallel tempering (Sec. II, Eq. (8)); each wave of 64 walkers holds floor(64/M)
// sets of M configurations (lanes g M .. g M + M - 1; the remaining lanes idle at slot 0, outside
// exchanges and bookkeeping), the row is the configuration's temperature slot, and after every
// sweep the slots (s, s+1) with s = t (mod 2) try an exchange. Temperatures are per realization.
// XT (multicanonical, no speculation): the table is expanded on chip to one row per level of
// the realization (rows outside the stored range repeat its edge rows, as the clamp would), so
// the row of a level is the level itself and the decision needs no clamp.
template <int L, bool SPEC, bool PT, bool XT = false, bool WS = false, bool SU = false>
__device__ __forceinline__ void sweep_wave(const SweepArgs& A, int wave) {
  using G = Geo<L>;
  using PW = typename G::PW;
  constexpr int NWP = G::NWP, Q = G::Q, N = G::N, H = G::H, FB = G::F;
  constexpr int NB = (G::BITS + 7) / 8;  // bytes of a plane-colour string
  constexpr int kZUnroll = L <= 6 ? L : 1;
  static_assert(!(PT && SPEC), "the tempering row does not depend on the decision");
  static_assert(!(XT && PT), "the expanded table is for the multicanonical form");
  static_assert(!(XT && SPEC) || WS, "the speculative form with the expanded table runs beside a generator wave");
  static_assert(!WS || XT, "the generator wave serves the expanded-table form");
  const int lane = (int)(threadIdx.x & 63u);
  const int r = A.wave_real[wave];
  const int wl = A.wave_wl[wave] + lane;
  const RealInfo& RI = A.reals[r];
  const int e_base = RI.e_base, walkers = RI.walkers, K = RI.K;
  const int row0 = (PT || XT) ? 0 : RI.row0, rows = PT ? A.pt_M : (XT ? K : RI.rows);
  const int e_bot = RI.e_bot, e_top = RI.e_top;
  const uint32_t real_id = RI.real_id;
  const int64_t gw = RI.walker_off + wl;

  // LDS (the kernel's only LDS, so it starts at address 0):
  //   [0, rows*32)        threshold table, each row permuted from u-order to m-order: entry j
  //                       holds the threshold of the step m = j (j < 4) or m = j - 8 (j > 4),
  //                       as th' of the decision (r <= th');
  //   tempering only      energies by slot, exchange decisions, exchange counters (3 x 256 B);
  //   then                the realization's couplings in the kernel layout;
  //   multicanonical only the launch's histogram over a window of levels around the table rows
  //   (all K levels where that costs no occupancy: walkers leave the rows in both directions,
  //   above the top where W is constant and below the lowest known level in the first rounds),
  //   flushed to HBM once at the end; levels outside the window are counted in HBM directly.
  const uint32_t sE = (uint32_t)rows * 32u, sD = sE + 256u, sAcc = sD + 256u;
  const uint32_t jbase = PT ? sAcc + 256u : sE;
  const uint32_t hbase = jbase + 4u * (uint32_t)jk_words(L);
  const int hlo = max(0, row0 - A.hist_margin), hn = A.hist_n;
  {
    const uint32_t* gt = A.tables + RI.table_off;
    for (int e = lane; e < rows * 8; e += 64) {
      const int jj = e & 7;
      const int u = jj < 4 ? 3 - jj : (jj == 4 ? 7 : 11 - jj);
      int gr = e >> 3;   // row of the stored table
      if constexpr (XT) gr = min(max(gr - RI.row0, 0), RI.rows - 1);
      const uint32_t v = PT ? A.pt_metro[((int64_t)r * kMaxReplicas + gr) * 8 + u] : gt[gr * 8 + u];
      const uint32_t vp = (v == 0xFFFFFFFFu) ? v : (v ? v - 1u : 0u);
      *(__attribute__((address_space(3))) uint32_t*)(uintptr_t)(e * 4) = vp;
    }
    const uint32_t* jg = A.jk + RI.jk_off;
    for (int e = lane; e < jk_words(L); e += 64) lds_store_i32(jbase + 4u * (uint32_t)e, (int)jg[e]);
  }
  if constexpr (PT) {
    lds_store_i32(sAcc + 4u * (uint32_t)lane, 0);
  } else {
    for (int e = lane; e < hn; e += 64) lds_store_i32(hbase + 4u * (uint32_t)e, 0);
  }
  __syncthreads();

  // walker state -> registers. One array per (colour, word) so that each stays small
  // enough to live in VGPRs under a dynamic plane index.
  uint32_t a00[L], a01[L], a02[L], a10[L], a11[L], a12[L];
  auto lat = [&](int c, int w) -> uint32_t* {
    return c == 0 ? (w == 0 ? a00 : w == 1 ? a01 : a02) : (w == 0 ? a10 : w == 1 ? a11 : a12);
  };
  static_assert(NWP <= 3, "plane-colour strings of at most 3 words");
  {
    const uint32_t* sp = A.spins + RI.spin_off + wl;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int w = 0; w < NWP; ++w)
#pragma unroll
        for (int z = 0; z < L; ++z) lat(c, w)[z] = sp[(int64_t)((c * L + z) * NWP + w) * walkers];
  }
  // tempering: this lane's set within the wave (floor(lane / M)), its first lane, its index in
  // the realization; lanes beyond the last whole set idle
  uint32_t pt_base = 0, pt_set = 0;
  bool pt_active = false;
  if constexpr (PT) {
    const uint32_t sw = __umulhi((uint32_t)lane, A.pt_minv);
    pt_active = sw < (uint32_t)A.pt_spw;
    pt_base = sw * (uint32_t)A.pt_M;
    pt_set = (uint32_t)(A.wave_wl[wave] >> 6) * (uint32_t)A.pt_spw + sw;
    asm volatile("" : "+v"(pt_base), "+v"(pt_set));
  }
  const int E0 = A.ws.E[gw];
  int E = E0;        // tempering: the energy, updated per attempt
  int slot = 0;      // tempering: the temperature slot
  int B;
  Track tr;
  TrackE te;
  if constexpr (PT) {
    slot = A.pt_slot[gw];
    B = slot * 32;
    te.Emin = A.ws.E_min[gw];
    te.state = A.ws.rt_state[gw];
    te.newmin = A.ws.new_min[gw];
    te.trips = 0;
    te.t_first = A.ws.t_first[gw];
    te.t_last = A.ws.t_last[gw];
  } else {
    B = ((E0 - e_base) / 4 - row0) * 32;
    tr.Bmin = ((A.ws.E_min[gw] - e_base) / 4 - row0) * 32;
    tr.state = A.ws.rt_state[gw];
    tr.newmin = A.ws.new_min[gw];
    tr.trips = 0;
    tr.t_first = A.ws.t_first[gw];
    tr.t_last = A.ws.t_last[gw];
  }

  const int Bmax = (rows - 1) * 32;
  const int Btop = (ceil_div4(e_top - e_base) - row0) * 32;    // E >= e_top  <=> B >= Btop
  const int Bbot = (floor_div4(e_bot - e_base) - row0) * 32;   // E <= e_bot  <=> B <= Bbot
  const int Bnm = (ceil_div4(e_bot - e_base) - 1 - row0) * 32; // E <  e_bot  <=> B <= Bnm
  Window win;
  if constexpr (!PT) win = make_window(tr.state, Bbot, Btop);
  int R = clamp_row(B, Bmax);   // the table row in use: B clamped to the stored rows
  int vBmax;                    // Bmax in a vector register (an operand of the decision sequence)
  asm volatile("v_mov_b32 %0, %1" : "=v"(vBmax) : "s"(Bmax));

  const uint32_t key0 = (uint32_t)A.walker_seed, key1 = (uint32_t)(A.walker_seed >> 32);
  // Round keys in VGPRs: uniform values, but keeping them out of the scalar file leaves room for
  // the per-plane coupling words and constants without spilling scalar registers. (Not needed
  // when a generator wave supplies the words.)
  PhiloxKeysV kv;
  if constexpr (!WS) kv = philox_round_keys_v(key0, key1);
  const uint32_t ctr3 = ((uint32_t)wl << 8) | (PT ? kTagPT : kTagAcc);

  // Level steps of the sites of block (c, z), a plane-colour string, from the other colour's
  // spins and the couplings: V[g8] holds, byte-interleaved, the three bits of m = 3 - u of eight
  // sites. The other colour does not change while colour c is updated, so the block after the
  // current one is prepared while the current one runs.
  auto block_steps = [&](int c, int z, uint32_t (&V)[NB]) __attribute__((always_inline)) {
    const int zp = (z + 1 == L) ? 0 : z + 1;
    const int zm = (z == 0) ? L - 1 : z - 1;
    uint32_t Cw[NWP], Ow[NWP], Pw[NWP], Mw[NWP];
#pragma unroll
    for (int w = 0; w < NWP; ++w) {
      Cw[w] = lat(c, w)[z];
      Ow[w] = lat(1 - c, w)[z];
      Pw[w] = lat(1 - c, w)[zp];
      Mw[w] = lat(1 - c, w)[zm];
    }
    const uint32_t jz = jbase + 4u * (uint32_t)((c * L + z) * 6 * NWP);
    uint32_t Jw[6][NWP];
    {
      // 6 NWP words, 8-byte aligned: read as pairs, all issued before the first use
      uint64_t jv[3 * NWP];
#pragma unroll
      for (int k = 0; k < 3 * NWP; ++k)
        jv[k] = *(const __attribute__((address_space(3))) uint64_t*)(uintptr_t)(jz + 8u * (uint32_t)k);
#pragma unroll
      for (int k = 0; k < 6; ++k)
#pragma unroll
        for (int w = 0; w < NWP; ++w) {
          const int e = k * NWP + w;
          Jw[k][w] = (uint32_t)(jv[e >> 1] >> (32 * (e & 1)));
        }
    }
    // flags: bit set <=> bond unsatisfied (S_i xor S_j xor [J = -1])
    const PW own = pack<L>(Cw), O = pack<L>(Ow), Zp = pack<L>(Pw), Zm = pack<L>(Mw);
    constexpr PW ALL = G::all_bits();
    const PW Yp = ((O >> G::F) | (O << (G::F * (L - 1)))) & ALL;
    const PW Ym = ((O << G::F) | (O >> (G::F * (L - 1)))) & ALL;
    const PW Xm1 = ((O << 1) & G::fields(1, G::H - 1)) | ((O >> (G::H - 1)) & G::fields(0, 1));
    const PW Xp1 = ((O >> 1) & G::fields(0, G::H - 1)) | ((O << (G::H - 1)) & G::fields(G::H - 1, 1));
    // rows whose sites have odd x (phi = 1) take their "other" x-neighbour at j+1
    const PW PHI = ((c + z) & 1) ? G::rows_of_parity(0) : G::rows_of_parity(1);
    const PW Xo = (Xp1 & PHI) | (Xm1 & ~PHI);
    const PW f1 = own ^ Zp ^ pack<L>(Jw[0]);
    const PW f2 = own ^ Zm ^ pack<L>(Jw[1]);
    const PW f3 = own ^ Yp ^ pack<L>(Jw[2]);
    const PW f4 = own ^ Ym ^ pack<L>(Jw[3]);
    const PW f5 = own ^ O ^ pack<L>(Jw[4]);
    const PW f6 = own ^ Xo ^ pack<L>(Jw[5]);
    // Bit-sliced u = f1 + ... + f6, delivered as the level step m = 3 - u in 3-bit two's
    // complement: m = (7 - u) ^ 4, i.e. bits (~u0, ~u1, u2).
    const PW s1 = f1 ^ f2 ^ f3, k1 = (f1 & f2) | (f3 & (f1 ^ f2));
    const PW s2 = f4 ^ f5 ^ f6, k2 = (f4 & f5) | (f6 & (f4 ^ f5));
    const PW t0 = s1 & s2;
    uint32_t m0[NWP], m1[NWP], m2[NWP];
    unpack<L>(~(s1 ^ s2), m0);
    unpack<L>(~(k1 ^ k2 ^ t0), m1);
    unpack<L>((k1 & k2) | (t0 & (k1 ^ k2)), m2);
    // Byte-interleave: V[g8] = (0, m0.byte, m1.byte, m2.byte). For the site at bit b of
    // that byte, (V & (0x01010100 << b)) * (2^(26-b) + 2^(19-b) + 2^(12-b)) puts its three
    // bits at 2^34, 2^35, 2^36 and every other partial product at another single bit
    // (no carries), so bits 2..4 of the high word are m & 7.
#pragma unroll
    for (int g8 = 0; g8 < NB; ++g8) {
      const int w = g8 >> 2;
      const uint32_t bsel = (uint32_t)(g8 & 3);
      // perm selector bytes: 0x0c -> 0x00; 0..3 pick src1 bytes, 4..7 pick src0 bytes
      const uint32_t lo = __builtin_amdgcn_perm(m1[w], m0[w], 0x0c00000cu | (bsel << 8) | ((4u + bsel) << 16));
      V[g8] = __builtin_amdgcn_perm(m2[w], lo, 0x00020100u | ((4u + bsel) << 24));
      asm volatile("" : "+v"(V[g8]));
    }
  };
  // m & 7 of site q of a block in bits 2..4 (sign at bit 4) of a product high word
  auto gather = [&](const uint32_t (&V)[NB], int q) __attribute__((always_inline)) -> uint32_t {
    const int y = q / H, j = q % H;
    const int p = y * FB + j, g8 = p >> 3, bb = p & 7;
    // (2^26 + 2^19 + 2^12) >> bb: eight distinct constants in all
    return __umulhi(V[g8] & (0x01010100u << bb), 0x04081000u >> bb);
  };
  auto lookup = [&](uint32_t hi, int Rv) __attribute__((always_inline)) -> uint32_t {
    // Rv is a multiple of 32 in [0, Bmax]; (hi & 0x1c) is 4 (m & 7)
    return *(const __attribute__((address_space(3))) uint32_t*)(uintptr_t)((hi & 0x1cu) | (uint32_t)Rv);
  };
  // Generator counter of group g (four sites) of block (c, z) in sweep t.
  auto group_ctr = [&](int c, int z, int g, uint64_t t) __attribute__((always_inline)) -> PhiloxRun {
    return PhiloxRun{((uint32_t)(c * L + z) << 8) | (uint32_t)g, (uint32_t)t, real_id, ctr3};
  };
  constexpr int NG = (Q + 3) / 4;
  // The generator runs one group ahead: pr holds the words of the next group of four sites, and
  // its rounds are spread over the attempts of the group before it (also across blocks, colours
  // and sweeps), so that they fill the wait for each threshold read.
  PhiloxRun pr{};
  if constexpr (!WS) {
    pr = group_ctr(0, 0, 0, A.t0);
    philox_rounds<0, 10>(pr, kv);
  }
  // Warp-specialized form: the words of block b sit in ring slot b mod 3; rw holds the next
  // group's words, read one group ahead.
  const uint32_t rbase = WS ? ws_ring_base(K, jk_words(L), hn) : 0u;
  auto ring = [&](uint32_t slot, int g) __attribute__((always_inline)) -> uint32_t {
    return rbase + slot * ws_slot_bytes<L>() + (uint32_t)(g * 64 + lane) * 16u;
  };
  uint32_t rslot = 0, rslot_n = 1;
  u32x4 rw{};
  if constexpr (WS) rw = lds_load_u32x4(ring(0, 0));

  for (uint32_t s = 0; s < A.n_sweeps; ++s) {
    const uint64_t t = A.t0 + s;
    const uint64_t tau0 = t * (uint64_t)N + 1u;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      uint32_t Vc[NB];
      block_steps(c, 0, Vc);
      // the colour's first threshold; later ones are read by the attempt before (multicanonical)
      // or one site ahead (tempering), across block ends
      uint32_t hi_cur = gather(Vc, 0);
      uint32_t th_fly = 0, addr_cur = 0;
      if constexpr (!SPEC || PT) th_fly = lookup(hi_cur, R);
      // small lattices: planes unrolled (static register indices); larger ones: a plane loop
      // whose dynamic index selects registers of the per-(colour, word) arrays
#pragma unroll kZUnroll
      for (int z = 0; z < L; ++z) {
        const bool has_next = z + 1 < L;
        uint32_t Vn[NB];
        if (has_next) block_steps(c, z + 1, Vn);
        uint32_t Cw[NWP];
#pragma unroll
        for (int w = 0; w < NWP; ++w) Cw[w] = lat(c, w)[z];
        const uint64_t tau_blk = tau0 + (uint64_t)(c * (N / 2) + z * Q);
        // Acceptance bits are shifted into F in site order, with a zero for every bit of a
        // field beyond the row's H sites, and applied to the plane-colour string once per word.
        uint32_t F = 0;
        // levels after each attempt since the last window check (kCheckGroups groups of four)
        constexpr int kCheckGroups = check_groups<L>();
        int Bq[4 * kCheckGroups];
        // speculative form: the pair for site 0 of the block is loaded at the block's start
        uint32_t p_rej = 0, p_acc = 0;
        int Racc_prev = R;
        if constexpr (SPEC && !PT) {
          hi_cur = gather(Vc, 0);
          p_rej = p_acc = lookup(hi_cur, R);
        }
#pragma unroll
        for (int g = 0; g < NG; ++g) {
          u32x4 rnd;
          if constexpr (WS) {
            // this group's words, and the read of the next group's (in this block, or the first
            // group of the next block, whose slot the generator filled before the last barrier)
            rnd = rw;
            rw = lds_load_u32x4(g + 1 < NG ? ring(rslot, g + 1) : ring(rslot_n, 0));
          } else {
            rnd = u32x4{{pr.c0, pr.c1, pr.c2, pr.c3}};
            // the next group: in this block, the next block, the other colour or the next sweep
            if (g + 1 < NG) pr = group_ctr(c, z, g + 1, t);
            else if (has_next) pr = group_ctr(c, z + 1, 0, t);
            else if (c == 0) pr = group_ctr(1, 0, 0, t);
            else pr = group_ctr(0, 0, 0, t + 1);
          }
          const int n_att = (4 * g + 4 <= Q) ? 4 : Q - 4 * g;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int q = 4 * g + i;
            if (q >= Q) break;
            const int y = q / H, j = q % H;
            const int p = y * FB + j, w = p >> 5;
            if constexpr (SPEC && !PT) {
              const uint32_t rc = rnd.v[i];
              if constexpr (!WS) {
                if (i == 0) {
                  if constexpr (SU) philox_rounds_u<0, 3>(pr, key0, key1);
                  else philox_rounds<0, 3>(pr, kv);
                }
                if (i == 1) philox_rounds<3, 5>(pr, kv);
                if (i == 2) philox_rounds<5, 8>(pr, kv);
                if (i == 3) philox_rounds<8, 10>(pr, kv);
              }
              // thresholds of site q+1 for both outcomes of q are loaded before q is decided; the
              // threshold of site q is picked from the pair loaded one site earlier
              const int Bacc = B + __builtin_amdgcn_sbfe((int)hi_cur, 2, 3) * 32;
              const int Racc = XT ? Bacc : clamp_row(Bacc, Bmax);
              uint32_t hi_next = 0, n_rej = 0, n_acc = 0;
              if (q + 1 < Q) {
                hi_next = gather(Vc, q + 1);
                n_rej = lookup(hi_next, R);
                n_acc = lookup(hi_next, Racc);
              }
              const uint32_t th_cur = (R == Racc_prev) ? p_acc : p_rej;
              accept_level_spec(rc, th_cur, Bacc, Racc, B, R, F);
              p_rej = n_rej;
              p_acc = n_acc;
              Racc_prev = Racc;
              hi_cur = hi_next;
            } else {
              // (1) the threshold of this site, read earlier (multicanonical: by the previous
              //     decision, at the address it computed; tempering: the row is fixed, so the
              //     next site's read is issued here, one attempt ahead)
              const uint32_t th = th_fly;
              uint32_t hi_next = 0;
              if (q + 1 < Q) hi_next = gather(Vc, q + 1);
              else if (has_next) hi_next = gather(Vn, 0);
              if constexpr (PT) {
                if (q + 1 < Q || has_next) th_fly = lookup(hi_next, R);
              }
              // (2) independent work: generator rounds of the next group. Empty volatile
              //     statements pin the order: they are ordered with the decision, and the
              //     rounds' outputs pass through the second one. The first takes only the words
              //     the round's products do not read: a VALU read of a register an asm statement
              //     wrote costs a wait state, and uniform words stay scalar.
              if constexpr (!WS) {
                // SU: rounds 0-2 act on a counter whose words 0..2 are still uniform, so their
                // uniform parts go to the scalar unit (pays where several waves share a SIMD and
                // scalar registers are not short)
                if constexpr (SU) {
                  if (i == 0) philox_rounds_u<0, 3>(pr, key0, key1);
                  if (i > 0) asm volatile("" : "+v"(pr.c1), "+v"(pr.c3));
                } else {
                  asm volatile("" : "+v"(pr.c1), "+v"(pr.c3));
                  if (i == 0) philox_rounds<0, 3>(pr, kv);
                }
                if (i == 1) philox_rounds<3, 5>(pr, kv);
                if (i == 2) philox_rounds<5, 8>(pr, kv);
                if (i == 3) philox_rounds<8, 10>(pr, kv);
              }
              const uint32_t rc = rnd.v[i];
              if constexpr (!WS) asm volatile("" : "+v"(pr.c0), "+v"(pr.c1), "+v"(pr.c2), "+v"(pr.c3));
              // (3) the decision, the next site's table address and (multicanonical) its read,
              //     issued before the bookkeeping and flips that follow
              if constexpr (PT) {
                accept_energy(rc, th, hi_cur, E, F);
              } else {
                if constexpr (XT) {
                  accept_level_xt(rc, th, hi_cur, hi_next, B, F, addr_cur);
                  R = B;
                } else {
                  accept_level(rc, th, hi_cur, hi_next, vBmax, B, R, F, addr_cur);
                }
                if (q + 1 < Q || has_next)
                  th_fly = *(const __attribute__((address_space(3))) uint32_t*)(uintptr_t)addr_cur;
              }
              hi_cur = hi_next;
            }
            Bq[4 * (g % kCheckGroups) + i] = B;
            // end of a row inside the word: zeros for the field's unused bits; end of the word
            // (or of the string): apply the flips
            const bool last_in_word = (q + 1 == Q) || (((((q + 1) / H) * FB + (q + 1) % H) >> 5) != w);
            if (last_in_word) {
              Cw[w] ^= __builtin_bitreverse32(F) >> (31 - (p & 31));
              F = 0;
            } else if (j == H - 1 && FB > H) {
              F <<= (FB - H);
            }
          }
          // a short last group: the generator rounds its missing attempts would have run
          if constexpr (!WS) {
            if (n_att == 1) philox_rounds<3, 10>(pr, kv);
            if (n_att == 2) philox_rounds<5, 10>(pr, kv);
            if (n_att == 3) philox_rounds<8, 10>(pr, kv);
          }
          if constexpr (!PT) {
            // Every kCheckGroups-th group (and at the block's end): the minimum and the
            // new-minimum flag from the lowest level since the last check; if an attempt since
            // then reached the bound the round-trip state waits for, replay those attempts'
            // state exactly.
            if (g % kCheckGroups == kCheckGroups - 1 || g + 1 == NG) {
              const int g0 = g - g % kCheckGroups;                 // first group since the check
              const int cnt = 4 * (g - g0) + n_att;                // attempts since the check
              int bmin = Bq[0], bmax = Bq[0];
#pragma unroll
              for (int k = 1; k < 4 * kCheckGroups; ++k) {
                if (k >= cnt) break;
                bmin = min(bmin, Bq[k]);
                bmax = max(bmax, Bq[k]);
              }
              tr.Bmin = min(tr.Bmin, bmin);
              tr.newmin = (bmin <= Bnm) ? 1 : tr.newmin;           // E < e_bot <=> B <= Bnm
              if (bmin < win.lo || bmax > win.hi) {
#pragma unroll
                for (int k = 0; k < 4 * kCheckGroups; ++k) {
                  if (k >= cnt) break;
                  track_attempt(tr, Bq[k], tau_blk + (uint64_t)(4 * g0 + k), Bbot, Btop);
                }
                win = make_window(tr.state, Bbot, Btop);
              }
            }
          }
        }
#pragma unroll
        for (int w = 0; w < NWP; ++w) lat(c, w)[z] = Cw[w];
        if constexpr (WS) {
          // this block's words are consumed: the generator may refill their slot
          __syncthreads();
          rslot = rslot_n;
          rslot_n = rslot_n == 2u ? 0u : rslot_n + 1u;
        }
        if (has_next) {
#pragma unroll
          for (int k = 0; k < NB; ++k) Vc[k] = Vn[k];
        }
      }
    }
    if constexpr (PT) {
      // end of the Metropolis phase: bookkeeping with stamp (t + 1) N, trace
      const int M = A.pt_M;
      const bool active = pt_active;
      if (active) track_energy(te, E, (t + 1u) * (uint64_t)N, e_bot, e_top);
      if (t - A.trace_t0 < (uint64_t)A.trace_cap && (uint64_t)(gw - A.trace_w0) < (uint64_t)A.trace_nw)
        A.trace[(gw - A.trace_w0) * A.trace_cap + (int64_t)(t - A.trace_t0)] = E;
      // exchange phase: slots (s, s+1), s = t (mod 2), of each set of M lanes
      const uint32_t base = pt_base;
      lds_store_i32(sE + 4u * (base + (uint32_t)slot), E);
      __syncthreads();
      const int par = (int)(t & 1u);
      const bool lower = active && ((slot & 1) == par) && (slot + 1 < M);
      const bool upper = active && (slot >= 1) && (((slot - 1) & 1) == par);
      int dec = 0;
      if (lower) {
        const int Eh = lds_load_i32(sE + 4u * (base + (uint32_t)slot + 1u));
        const int d = (Eh - E) / 4;   // energies of one realization share their residue mod 4
        const uint32_t th = pt_swap_threshold(A.pt_q[(int64_t)r * kMaxReplicas + slot], d);
        const uint32_t set = pt_set;   // set index within the realization
        const u32x4 rr = philox4x32_10_vk((uint32_t)(slot >> 2), (uint32_t)t, real_id, (set << 8) | kTagSwap, kv);
        const int k4 = slot & 3;
        const uint32_t rw = k4 == 0 ? rr.v[0] : k4 == 1 ? rr.v[1] : k4 == 2 ? rr.v[2] : rr.v[3];
        dec = min(rw, 0xFFFFFFFEu) < th ? 1 : 0;
        lds_store_i32(sD + 4u * (base + (uint32_t)slot), dec);
        if (dec) {
          const uint32_t ca = sAcc + 4u * (base + (uint32_t)slot);
          lds_store_i32(ca, lds_load_i32(ca) + 1);
        }
      }
      __syncthreads();
      int nslot = slot;
      if (lower && dec) nslot = slot + 1;
      if (upper && lds_load_i32(sD + 4u * (base + (uint32_t)slot - 1u))) nslot = slot - 1;
      slot = nslot;
      B = slot * 32;
      R = B;
      __syncthreads();
    } else {
      // end of sweep: histogram (on chip) and trace
      const int k = (B >> 5) + row0;
      const uint32_t kh = (uint32_t)(k - hlo);
      if (kh < (uint32_t)hn && k < K)
        __hip_atomic_fetch_add((__attribute__((address_space(3))) uint32_t*)(uintptr_t)(hbase + 4u * kh), 1u,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      else if ((uint32_t)k < (uint32_t)K)  // always true for exact energies
        atomicAdd(A.hist + RI.level_off + k, 1ULL);
      if (t - A.trace_t0 < (uint64_t)A.trace_cap && (uint64_t)(gw - A.trace_w0) < (uint64_t)A.trace_nw)
        A.trace[(gw - A.trace_w0) * A.trace_cap + (int64_t)(t - A.trace_t0)] = e_base + 4 * k;
    }
  }

  // registers -> walker state
  {
    uint32_t* sp = A.spins + RI.spin_off + wl;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int w = 0; w < NWP; ++w)
#pragma unroll
        for (int z = 0; z < L; ++z) sp[(int64_t)((c * L + z) * NWP + w) * walkers] = lat(c, w)[z];
  }
  if constexpr (PT) {
    A.ws.E[gw] = E;
    A.ws.E_min[gw] = te.Emin;
    A.ws.rt_state[gw] = te.state;
    A.ws.new_min[gw] = te.newmin;
    A.ws.rt_count[gw] += te.trips;
    A.ws.t_first[gw] = te.t_first;
    A.ws.t_last[gw] = te.t_last;
    A.pt_slot[gw] = slot;
    // exchange counters of the pairs (s, s+1) of this lane's set, s = lane index in the set
    const int M = A.pt_M;
    const int cidx = (int)((uint32_t)lane - pt_base);
    if (pt_active && cidx < M - 1)   // global set index: walker offsets of realizations are multiples of 64
      A.pt_acc[(int64_t)(RI.walker_off / 64 * A.pt_spw + pt_set) * (M - 1) + cidx] +=
          (uint64_t)lds_load_i32(sAcc + 4u * (uint32_t)lane);
  } else {
    // the launch's histogram counts (at most 64 walkers x 2^20 sweeps per level)
    __syncthreads();
    for (int e = lane; e < hn; e += 64) {
      const uint32_t c = (uint32_t)lds_load_i32(hbase + 4u * (uint32_t)e);
      if (c) atomicAdd(A.hist + RI.level_off + hlo + e, (unsigned long long)c);   // c > 0: hlo + e < K
    }
    A.ws.E[gw] = e_base + 4 * ((B >> 5) + row0);
    A.ws.E_min[gw] = e_base + 4 * ((tr.Bmin >> 5) + row0);
    A.ws.rt_state[gw] = tr.state;
    A.ws.new_min[gw] = tr.newmin;
    A.ws.rt_count[gw] += tr.trips;
    A.ws.t_first[gw] = tr.t_first;
    A.ws.t_last[gw] = tr.t_last;
  }
}

// The generator wave of the warp-specialized form: the words of every group of every block of
// the launch (blocks in sweep order: sweep, colour, plane), two blocks ahead of the sampling
// wave. It meets the sampling wave at the same barriers: after the tables are staged, at the end
// of every block, before the histogram flush.
template <int L>
__device__ __forceinline__ void generate_words(const SweepArgs& A, int wave) {
  constexpr int Q = Geo<L>::Q, NG = (Q + 3) / 4;
  const int lane = (int)(threadIdx.x & 63u);
  const RealInfo& RI = A.reals[A.wave_real[wave]];
  const uint32_t ctr3 = ((uint32_t)(A.wave_wl[wave] + lane) << 8) | kTagAcc, real_id = RI.real_id;
  const uint32_t key0 = (uint32_t)A.walker_seed, key1 = (uint32_t)(A.walker_seed >> 32);
  const uint32_t rbase = ws_ring_base(RI.K, jk_words(L), A.hist_n);
  // blocks in the sampling wave's order; (t, cz = c L + z) names the block to be written next
  const uint32_t nb = (uint32_t)A.n_sweeps * 2u * (uint32_t)L;   // at most 2^20 sweeps per launch
  uint32_t t = (uint32_t)A.t0, cz = 0;
  auto advance = [&]() __attribute__((always_inline)) {
    if (++cz == 2u * (uint32_t)L) {
      cz = 0;
      ++t;
    }
  };
  auto fill = [&](uint32_t slot) __attribute__((always_inline)) {
    for (int g = 0; g < NG; ++g) {
      const u32x4 w = philox4x32_10_u((cz << 8) | (uint32_t)g, t, real_id, ctr3, key0, key1);
      lds_store_u32x4(rbase + slot * ws_slot_bytes<L>() + (uint32_t)(g * 64 + lane) * 16u, w);
    }
  };
  if (nb > 0u) fill(0u);
  advance();
  if (nb > 1u) fill(1u);
  advance();
  __syncthreads();   // tables staged, blocks 0 and 1 written
  uint32_t slot = 2;
  for (uint32_t b = 0; b < nb; ++b) {
    if (b + 2u < nb) fill(slot);   // block b + 2
    advance();
    slot = slot == 2u ? 0u : slot + 1u;
    __syncthreads();   // the sampling wave has finished block b
  }
  __syncthreads();     // before the sampling wave's histogram flush
}

template <int L, bool SPEC>
__global__ void __launch_bounds__(128) k_sweeps_ws(SweepArgs A) {
  extern __shared__ uint32_t stab[];  // addressed from LDS address 0
  (void)stab;
  // the role is uniform per wave: a scalar branch, so that each wave meets only its own barriers
  const int role = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  if (role == 0) {
    // the sampling wave's decisions form the critical chain: its instructions go first
    __builtin_amdgcn_s_setprio(3);
    sweep_wave<L, SPEC, false, true, true>(A, (int)blockIdx.x);
  } else {
    generate_words<L>(A, (int)blockIdx.x);
  }
}

template <int L, bool SPEC, bool PT, bool XT>
__global__ void __launch_bounds__(64) k_sweeps(SweepArgs A) {
  extern __shared__ uint32_t stab[];  // addressed from LDS address 0 by sweep_wave
  (void)stab;
  // scalar uniform rounds for the compact and tempering forms (usually several waves per SIMD),
  // except the L = 6 tempering form, where they cost a resident wave (139 against 125 VGPRs)
  sweep_wave<L, SPEC, PT, XT, false, !XT && !(PT && L == 6)>(A, (int)blockIdx.x);
}

// Persistent multicanonical launch over a batch of mixed lattice sizes: each workgroup takes
// work items (one wave of walkers for this launch's sweeps) from a global counter until the
// queue is empty. The queue lists waves longest-first (by N), so the last items to start are
// the cheapest ones. Results do not depend on which workgroup runs which item.
// MAXL: the largest lattice the launch's items have (a launch over small lattices only holds
// fewer registers per wave, so more waves stay resident). SOLO: the wave claims the whole
// register file of its SIMD (all 256 accumulation registers besides its own), so no other wave
// shares that SIMD's issue slots while it runs; for the largest lattices, whose serial chains
// bound the batch.
template <bool SPEC, int MAXL, bool SOLO = false>
__global__ void __launch_bounds__(64) k_sweeps_queue(SweepArgs A, const int32_t* __restrict__ order, int n_items,
                                                     uint32_t* __restrict__ counter) {
  extern __shared__ uint32_t stab[];
  (void)stab;
  if constexpr (SOLO) asm volatile("" ::: "a255");
  for (;;) {
    __syncthreads();  // the previous item's table reads are done before the next table is loaded
    int item = 0;
    if (threadIdx.x == 0) item = (int)atomicAdd(counter, 1u);
    item = __shfl(item, 0, 64);
    if (item >= n_items) break;
    const int wave = order[item];
    switch (A.reals[A.wave_real[wave]].L) {
      case 2: sweep_wave<2, SPEC, false>(A, wave); break;
      case 4: if constexpr (MAXL >= 4) sweep_wave<4, SPEC, false>(A, wave); break;
      case 6: if constexpr (MAXL >= 6) sweep_wave<6, SPEC, false>(A, wave); break;
      case 8: if constexpr (MAXL >= 8) sweep_wave<8, SPEC, false>(A, wave); break;
      case 10: if constexpr (MAXL >= 10) sweep_wave<10, SPEC, false>(A, wave); break;
      case 12: if constexpr (MAXL >= 12) sweep_wave<12, SPEC, false>(A, wave); break;
      default: break;
    }
  }
}

// The exchange thresholds the sweep kernel uses for realization r, for inspection: [s][d - 1]
// for d = 1..D.
__global__ void k_pt_swap_table(const double* q, int r, int M, int D, uint32_t* swap) {
  const double* qr = q + (int64_t)r * kMaxReplicas;
  for (int f = blockIdx.x * blockDim.x + threadIdx.x; f < (M - 1) * D; f += gridDim.x * blockDim.x)
    swap[f] = pt_swap_threshold(qr[f / D], f % D + 1);
}

hipError_t launch_pt_swap_table(const double* q, int r, int M, int D, uint32_t* swap, hipStream_t s) {
  if (M < 2 || M > kMaxReplicas || D < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pt_swap_table, dim3(64), dim3(256), 0, s, q, r, M, D, swap);
  return hipGetLastError();
}

__global__ void k_fill_u32(uint32_t* p, int n, uint32_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Name of the sweep kernel the last launch on this host thread used (for reports).
static thread_local char g_last_kernel[48] = "none";
const char* last_sweep_kernel() { return g_last_kernel; }
void note_partitioned_launch(bool spec) {
  snprintf(g_last_kernel, sizeof(g_last_kernel), "%s_solo", spec ? "k_sweeps_queue_spec" : "k_sweeps_queue");
}
static void note_kernel(const char* form, int L) { snprintf(g_last_kernel, sizeof(g_last_kernel), "%s<%d>", form, L); }

template <int L, bool SPEC, bool PT, bool XT = false>
static hipError_t launch_LS(const SweepArgs& a, int n_waves, size_t lds_bytes, hipStream_t s) {
  // The kernel addresses its dynamic LDS block from address 0, which is only valid
  // when the compiler placed nothing else in LDS.
  static int checked = 0;
  if (!checked) {
    hipFuncAttributes attr;
    hipError_t e = hipFuncGetAttributes(&attr, reinterpret_cast<const void*>(&k_sweeps<L, SPEC, PT, XT>));
    if (e != hipSuccess) return e;
    if (attr.sharedSizeBytes != 0) return hipErrorInvalidKernelFile;
    checked = 1;
  }
  note_kernel(PT ? "k_sweeps_pt" : SPEC ? "k_sweeps_spec" : XT ? "k_sweeps_xt" : "k_sweeps", L);
  hipLaunchKernelGGL((k_sweeps<L, SPEC, PT, XT>), dim3(n_waves), dim3(64), lds_bytes, s, a);
  return hipGetLastError();
}

// Levels kept on chip below the table rows and above them when the histogram is a window.
constexpr int kHistMargin = 64;

// The histogram's extent for a launch: every level of the realization when that leaves as many
// workgroups resident per CU as the window would (capped at the ones the launch needs), else the
// window [row0 - kHistMargin, row0 + rows + kHistMargin).
struct HistPlan {
  int margin, n;
  size_t lds;
};

static HistPlan plan_hist(const void* f, size_t base_lds, int rows, int K, int want_blocks, int mode) {
  const HistPlan full{K, K, base_lds + (size_t)K * 4};
  const int nw = std::min(K, rows + 2 * kHistMargin);
  const HistPlan win{kHistMargin, nw, base_lds + (size_t)nw * 4};
  if (mode == 1) return win;
  if (mode == 2) return full;
  if (mode == 3) return HistPlan{0, std::min(K, rows), base_lds + (size_t)std::min(K, rows) * 4};
  int occ_full = 0, occ_win = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_full, f, 64, full.lds) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_win, f, 64, win.lds) != hipSuccess)
    return win;
  return occ_full >= std::min(occ_win, want_blocks) ? full : win;
}

template <int L, bool SPEC>
static hipError_t launch_ws(const SweepArgs& a, int n_waves, size_t lds_bytes, hipStream_t s) {
  static int checked = 0;
  if (!checked) {
    hipFuncAttributes attr;
    hipError_t e = hipFuncGetAttributes(&attr, reinterpret_cast<const void*>(&k_sweeps_ws<L, SPEC>));
    if (e != hipSuccess) return e;
    if (attr.sharedSizeBytes != 0) return hipErrorInvalidKernelFile;
    checked = 1;
  }
  note_kernel(SPEC ? "k_sweeps_ws_spec" : "k_sweeps_ws", L);
  hipLaunchKernelGGL((k_sweeps_ws<L, SPEC>), dim3(n_waves), dim3(128), lds_bytes, s, a);
  return hipGetLastError();
}

// ws_mode (expanded-table launches): 0 automatic -- the generator wave when the launch has at
// most one wave of walkers per SIMD (4 per CU) and all its workgroups stay resident -- 1 never,
// 2 always (when the expanded table is used).
template <int L>
static hipError_t launch_L(SweepArgs a, int n_waves, int lds_rows, int hist_levels, int n_cu, int hist_mode,
                           int ws_mode, bool spec, bool pt, hipStream_t s) {
  const size_t jb = (size_t)jk_words(L) * 4;
  if (pt) return launch_LS<L, false, true>(a, n_waves, (size_t)a.pt_M * 32 + 3 * 256 + jb, s);
  const void* f = spec ? reinterpret_cast<const void*>(&k_sweeps<L, true, false, false>)
                       : reinterpret_cast<const void*>(&k_sweeps<L, false, false, false>);
  const int want = (n_waves + n_cu - 1) / std::max(n_cu, 1);
  const HistPlan h = plan_hist(f, (size_t)lds_rows * 32 + jb, lds_rows, hist_levels, want, hist_mode);   // table, couplings
  if (hist_mode == 0) {
    // the expanded table (and every level of the histogram) when it costs no resident workgroups
    const void* fx = reinterpret_cast<const void*>(&k_sweeps<L, false, false, true>);
    const size_t lds_x = (size_t)hist_levels * 32 + jb + (size_t)hist_levels * 4;
    int occ_x = 0, occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_x, fx, 64, lds_x) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, f, 64, h.lds) == hipSuccess && occ_x >= std::min(occ, want)) {
      if (ws_mode != 1) {
        const size_t lds_w = (size_t)ws_ring_base(hist_levels, jk_words(L), hist_levels) + 3 * (size_t)ws_slot_bytes<L>();
        const void* fw = spec ? reinterpret_cast<const void*>(&k_sweeps_ws<L, true>)
                              : reinterpret_cast<const void*>(&k_sweeps_ws<L, false>);
        int occ_w = 0;
        const bool fits = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_w, fw, 128, lds_w) == hipSuccess &&
                          occ_w >= want;
        if (ws_mode == 2 ? occ_w >= 1 : (fits && n_waves <= 4 * n_cu)) {
          a.hist_margin = hist_levels;
          a.hist_n = hist_levels;
          return spec ? launch_ws<L, true>(a, n_waves, lds_w, s) : launch_ws<L, false>(a, n_waves, lds_w, s);
        }
      }
      if (!spec) {
        a.hist_margin = hist_levels;
        a.hist_n = hist_levels;
        return launch_LS<L, false, false, true>(a, n_waves, lds_x, s);
      }
    }
  }
  a.hist_margin = h.margin;
  a.hist_n = h.n;
  return spec ? launch_LS<L, true, false>(a, n_waves, h.lds, s) : launch_LS<L, false, false>(a, n_waves, h.lds, s);
}

static hipError_t launch_any(int L, const SweepArgs& a, int n_waves, int lds_rows, int hist_levels, int n_cu,
                             int hist_mode, int ws_mode, bool spec, bool pt, hipStream_t s) {
  switch (L) {
    case 2: return launch_L<2>(a, n_waves, lds_rows, hist_levels, n_cu, hist_mode, ws_mode, spec, pt, s);
    case 4: return launch_L<4>(a, n_waves, lds_rows, hist_levels, n_cu, hist_mode, ws_mode, spec, pt, s);
    case 6: return launch_L<6>(a, n_waves, lds_rows, hist_levels, n_cu, hist_mode, ws_mode, spec, pt, s);
    case 8: return launch_L<8>(a, n_waves, lds_rows, hist_levels, n_cu, hist_mode, ws_mode, spec, pt, s);
    case 10: return launch_L<10>(a, n_waves, lds_rows, hist_levels, n_cu, hist_mode, ws_mode, spec, pt, s);
    case 12: return launch_L<12>(a, n_waves, lds_rows, hist_levels, n_cu, hist_mode, ws_mode, spec, pt, s);
    default: return hipErrorInvalidValue;
  }
}

bool sweep_supported(int L) { return L >= 2 && L <= kMaxL && (L % 2) == 0; }

hipError_t launch_muca_sweeps(int L, const SweepArgs& a, int n_waves, int lds_rows, int hist_levels, int n_cu,
                              int hist_mode, int ws_mode, bool spec, hipStream_t s) {
  return launch_any(L, a, n_waves, lds_rows, hist_levels, n_cu, hist_mode, ws_mode, spec, false, s);
}

// The compiled queue forms: MAXL 8, 10 or 12, and the SIMD-exclusive form (MAXL 12).
static int queue_maxl(int maxl) { return maxl <= 8 ? 8 : maxl <= 10 ? 10 : kMaxL; }

template <bool SPEC>
static const void* queue_kernel_S(int maxl, bool solo) {
  if (solo) return reinterpret_cast<const void*>(&k_sweeps_queue<SPEC, kMaxL, true>);
  switch (queue_maxl(maxl)) {
    case 8: return reinterpret_cast<const void*>(&k_sweeps_queue<SPEC, 8>);
    case 10: return reinterpret_cast<const void*>(&k_sweeps_queue<SPEC, 10>);
    default: return reinterpret_cast<const void*>(&k_sweeps_queue<SPEC, kMaxL>);
  }
}

static const void* queue_kernel(bool spec, int maxl, bool solo) {
  return spec ? queue_kernel_S<true>(maxl, solo) : queue_kernel_S<false>(maxl, solo);
}

template <bool SPEC, int MAXL, bool SOLO>
static hipError_t launch_queue_S(const SweepArgs& a, const int32_t* order, int n_items, uint32_t* counter, int grid,
                                 size_t lds_bytes, hipStream_t s) {
  static int checked = 0;
  if (!checked) {
    hipFuncAttributes attr;
    hipError_t e = hipFuncGetAttributes(&attr, reinterpret_cast<const void*>(&k_sweeps_queue<SPEC, MAXL, SOLO>));
    if (e != hipSuccess) return e;
    if (attr.sharedSizeBytes != 0) return hipErrorInvalidKernelFile;
    checked = 1;
  }
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, counter, 1, 0u);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  snprintf(g_last_kernel, sizeof(g_last_kernel), "%s", SPEC ? "k_sweeps_queue_spec" : "k_sweeps_queue");
  hipLaunchKernelGGL((k_sweeps_queue<SPEC, MAXL, SOLO>), dim3(grid), dim3(64), lds_bytes, s, a, order, n_items,
                     counter);
  return hipGetLastError();
}

template <bool SPEC>
static hipError_t launch_queue_M(int maxl, bool solo, const SweepArgs& a, const int32_t* order, int n_items,
                                 uint32_t* counter, int grid, size_t lds_bytes, hipStream_t s) {
  if (solo) return launch_queue_S<SPEC, kMaxL, true>(a, order, n_items, counter, grid, lds_bytes, s);
  switch (queue_maxl(maxl)) {
    case 8: return launch_queue_S<SPEC, 8, false>(a, order, n_items, counter, grid, lds_bytes, s);
    case 10: return launch_queue_S<SPEC, 10, false>(a, order, n_items, counter, grid, lds_bytes, s);
    default: return launch_queue_S<SPEC, kMaxL, false>(a, order, n_items, counter, grid, lds_bytes, s);
  }
}

// LDS of the persistent kernel: the largest table, the couplings of the largest lattice and the
// histogram planned for the largest table and level count of the launch's items.
static HistPlan queue_plan(bool spec, int maxl, bool solo, int lds_rows, int hist_levels, int want_blocks,
                           int mode) {
  const int jl = solo ? kMaxL : queue_maxl(maxl);
  return plan_hist(queue_kernel(spec, maxl, solo), (size_t)lds_rows * 32 + (size_t)jk_words(jl) * 4, lds_rows,
                   hist_levels, want_blocks, mode);
}

int queue_blocks_per_cu(bool spec, int lds_rows, int hist_levels, int hist_mode, int maxl, bool solo) {
  int n = 0;
  const void* k = queue_kernel(spec, maxl, solo);
  const HistPlan h = queue_plan(spec, maxl, solo, lds_rows, hist_levels, 1 << 20, hist_mode);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, 64, h.lds) != hipSuccess) return 0;
  return n;
}

hipError_t launch_muca_queue(SweepArgs a, const int32_t* order, int n_items, uint32_t* counter, int grid, int n_cu,
                             int lds_rows, int hist_levels, int hist_mode, bool spec, hipStream_t s, int maxl,
                             bool solo) {
  if (grid < 1 || n_items < 0 || maxl < 2 || maxl > kMaxL) return hipErrorInvalidValue;
  const HistPlan h =
      queue_plan(spec, maxl, solo, lds_rows, hist_levels, (grid + n_cu - 1) / std::max(n_cu, 1), hist_mode);
  a.hist_margin = h.margin;
  a.hist_n = h.n;
  return spec ? launch_queue_M<true>(maxl, solo, a, order, n_items, counter, grid, h.lds, s)
              : launch_queue_M<false>(maxl, solo, a, order, n_items, counter, grid, h.lds, s);
}

// A short bounded wait (six sleeps of about 8k cycles each) on one stream, so that a launch
// queued on another stream at the same moment is placed on the CUs first.
__global__ void k_hold() {
  for (int i = 0; i < 6; ++i) __builtin_amdgcn_s_sleep(127);
}

hipError_t launch_hold(hipStream_t s) {
  hipLaunchKernelGGL(k_hold, dim3(1), dim3(64), 0, s);
  return hipGetLastError();
}

hipError_t launch_pt_sweeps(int L, const SweepArgs& a, int n_waves, hipStream_t s) {
  if (a.pt_M < 2 || a.pt_M > kMaxReplicas || a.pt_spw != 64 / a.pt_M ||
      a.pt_minv != 0xFFFFFFFFu / (uint32_t)a.pt_M + 1u)
    return hipErrorInvalidValue;
  return launch_any(L, a, n_waves, 1, 0, 1, 0, 1, false, true, s);
}

}  // namespace nfm
