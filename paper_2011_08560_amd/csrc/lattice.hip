// Lattice, coupling and spin kernels of libnfm: disorder draw (Sec. II), the
// ABI <-> kernel layout conversions, initial spins, the energy of Eq. (1) and
// the per-realization reduction of walker statistics (Sec. III).
#include "kernels.hpp"
#include "philox.hpp"

namespace nfm {

// ---------------------------------------------------------------------------------------------
// Kernel-layout position of site (x, y, z): colour c = (x+y+z)&1, plane z, field y, bit j = x>>1.
__device__ __forceinline__ void site_pos(int L, int x, int y, int z, int* word, int* bit) {
  const int F = field_bits(L), NWP = plane_words(L);
  const int c = (x + y + z) & 1;
  const int p = y * F + (x >> 1);
  *word = (c * L + z) * NWP + (p >> 5);
  *bit = p & 31;
}

__device__ __forceinline__ int abi_j(const uint32_t* jabi, int JW, int d, int i) {
  return (jabi[d * JW + (i >> 5)] >> (i & 31)) & 1;  // 1 <=> J = -1
}

// Sec. II: 3V couplings, each -1 with probability 1/2. Stream bit c = d*N + i is bit c%32 of
// output[m & 3] of Philox counter (m >> 2, id, 0, TAG_J), m = c/32, key = disorder seed.
__global__ void k_gen_couplings(const RealInfo* __restrict__ reals, uint32_t* __restrict__ jabi_all,
                                uint32_t key0, uint32_t key1) {
  const RealInfo ri = reals[blockIdx.x];
  const int JW = abi_plane_words(ri.N);
  uint32_t* jabi = jabi_all + ri.jabi_off;
  for (int t = threadIdx.x; t < 3 * JW; t += blockDim.x) {
    const int d = t / JW, w = t % JW;
    uint32_t word = 0;
    for (int b = 0; b < 32; ++b) {
      const int i = w * 32 + b;
      if (i >= ri.N) break;
      const uint32_t c = (uint32_t)(d * ri.N + i);
      const uint32_t m = c >> 5;
      const u32x4 r = philox4x32_10(m >> 2, ri.real_id, 0u, kTagJ, key0, key1);
      word |= ((r.v[m & 3] >> (c & 31)) & 1u) << b;
    }
    jabi[t] = word;
  }
}

// ABI couplings -> kernel layout, plus n_minus, e_base and K of the realization.
// Kernel layout of (c, z), field y, bit j (site x = 2j + phi, phi = (c+y+z)&1):
//   0 Jz(x,y,z)  1 Jz(x,y,z-1)  2 Jy(x,y,z)  3 Jy(x,y-1,z)
//   4 Jx of the partner bond (phi=0: bond x--x+1 owned by x; phi=1: bond x-1--x owned by x-1)
//   5 Jx of the other bond   (phi=0: bond x-1--x owned by x-1; phi=1: bond x--x+1 owned by x)
__global__ void k_pack_couplings(RealInfo* __restrict__ reals, const uint32_t* __restrict__ jabi_all,
                                 uint32_t* __restrict__ jk_all) {
  RealInfo* rp = reals + blockIdx.x;
  const int L = rp->L, N = rp->N, F = field_bits(L), NWP = plane_words(L), H = L / 2;
  const int JW = abi_plane_words(N);
  const uint32_t* jabi = jabi_all + rp->jabi_off;
  uint32_t* jk = jk_all + rp->jk_off;
  const int total = 2 * L * 6 * NWP;
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int w = t % NWP;
    const int kind = (t / NWP) % 6;
    const int cz = t / (6 * NWP);
    const int c = cz / L, z = cz % L;
    uint32_t word = 0;
    for (int b = 0; b < 32; ++b) {
      const int p = w * 32 + b;
      const int y = p / F, j = p % F;
      if (y >= L || j >= H) continue;
      const int phi = (c + y + z) & 1;
      const int x = 2 * j + phi;
      const int xm = (x + L - 1) % L, ym = (y + L - 1) % L, zm = (z + L - 1) % L;
      auto idx = [L](int xx, int yy, int zz) { return xx + L * yy + L * L * zz; };
      int bit = 0;
      switch (kind) {
        case 0: bit = abi_j(jabi, JW, 2, idx(x, y, z)); break;
        case 1: bit = abi_j(jabi, JW, 2, idx(x, y, zm)); break;
        case 2: bit = abi_j(jabi, JW, 1, idx(x, y, z)); break;
        case 3: bit = abi_j(jabi, JW, 1, idx(x, ym, z)); break;
        case 4: bit = phi == 0 ? abi_j(jabi, JW, 0, idx(x, y, z)) : abi_j(jabi, JW, 0, idx(xm, y, z)); break;
        default: bit = phi == 0 ? abi_j(jabi, JW, 0, idx(xm, y, z)) : abi_j(jabi, JW, 0, idx(x, y, z)); break;
      }
      word |= (uint32_t)bit << b;
    }
    jk[t] = word;
  }
  // n_minus over the 3N valid bits
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  int local = 0;
  for (int t = threadIdx.x; t < 3 * JW; t += blockDim.x) {
    const int w = t % JW;
    uint32_t v = jabi[t];
    const int valid = N - w * 32;
    if (valid < 32) v &= (1u << valid) - 1u;
    local += __popc(v);
  }
  atomicAdd(&cnt, local);
  __syncthreads();
  if (threadIdx.x == 0) {
    rp->n_minus = cnt;
    rp->e_base = -3 * N + 2 * (cnt & 1);
    rp->K = (3 * N - rp->e_base) / 4 + 1;
  }
}

// Initial spins: bit i of walker w is bit i%32 of output[m & 3] of counter
// (m >> 2, 0, id, (w << 8) | TAG_SPIN), m = i/32, key = walker seed; bit set <=> S = -1.
__global__ void k_gen_spins(const RealInfo* __restrict__ reals, int32_t r0, int32_t nr,
                            uint32_t* __restrict__ spins, uint32_t key0, uint32_t key1) {
  const int r = r0 + blockIdx.y;
  if (blockIdx.y >= (unsigned)nr) return;
  const RealInfo ri = reals[r];
  const int wl = blockIdx.x * blockDim.x + threadIdx.x;
  if (wl >= ri.walkers) return;
  const int L = ri.L, WPW = walker_words(L);
  uint32_t* base = spins + ri.spin_off;
  for (int k = 0; k < WPW; ++k) base[(int64_t)k * ri.walkers + wl] = 0;
  for (int i = 0; i < ri.N; ++i) {
    const uint32_t m = (uint32_t)i >> 5;
    const u32x4 rr = philox4x32_10(m >> 2, 0u, ri.real_id, ((uint32_t)wl << 8) | kTagSpin, key0, key1);
    const uint32_t bit = (rr.v[m & 3] >> (i & 31)) & 1u;
    int word, b;
    site_pos(L, i % L, (i / L) % L, i / (L * L), &word, &b);
    base[(int64_t)word * ri.walkers + wl] |= bit << b;
  }
}

// int8 spins (walker-major, N each) <-> kernel layout for walkers [wl0, wl0+count) of realization r.
__global__ void k_pack_spins(const RealInfo* __restrict__ reals, int32_t r, int32_t wl0, int32_t count,
                             const int8_t* __restrict__ src, uint32_t* __restrict__ spins) {
  const RealInfo ri = reals[r];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const int wl = wl0 + t, L = ri.L, WPW = walker_words(L);
  uint32_t* base = spins + ri.spin_off;
  for (int k = 0; k < WPW; ++k) base[(int64_t)k * ri.walkers + wl] = 0;
  for (int i = 0; i < ri.N; ++i) {
    int word, b;
    site_pos(L, i % L, (i / L) % L, i / (L * L), &word, &b);
    if (src[(int64_t)t * ri.N + i] < 0) base[(int64_t)word * ri.walkers + wl] |= 1u << b;
  }
}

__global__ void k_unpack_spins(const RealInfo* __restrict__ reals, int32_t r, int32_t wl0, int32_t count,
                               const uint32_t* __restrict__ spins, int8_t* __restrict__ dst) {
  const RealInfo ri = reals[r];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const int wl = wl0 + t, L = ri.L;
  const uint32_t* base = spins + ri.spin_off;
  for (int i = 0; i < ri.N; ++i) {
    int word, b;
    site_pos(L, i % L, (i / L) % L, i / (L * L), &word, &b);
    dst[(int64_t)t * ri.N + i] = ((base[(int64_t)word * ri.walkers + wl] >> b) & 1u) ? -1 : 1;
  }
}

// Eq. (1): E = -sum over sites and forward directions of J S_i S_{i+e_d}. Resets the walker's
// bookkeeping (E_min = E, no round trips, no new minimum).
__global__ void k_energy(const RealInfo* __restrict__ reals, const uint32_t* __restrict__ jabi_all,
                         const uint32_t* __restrict__ spins, WalkerState ws) {
  const RealInfo ri = reals[blockIdx.y];
  const int wl = blockIdx.x * blockDim.x + threadIdx.x;
  if (wl >= ri.walkers) return;
  const int L = ri.L, N = ri.N, JW = abi_plane_words(N);
  const uint32_t* jabi = jabi_all + ri.jabi_off;
  const uint32_t* base = spins + ri.spin_off;
  auto spin_bit = [&](int x, int y, int z) {
    int word, b;
    site_pos(L, x, y, z, &word, &b);
    return (int)((base[(int64_t)word * ri.walkers + wl] >> b) & 1u);
  };
  int E = 0;
  for (int i = 0; i < N; ++i) {
    const int x = i % L, y = (i / L) % L, z = i / (L * L);
    const int s = spin_bit(x, y, z);
    const int nb[3] = {spin_bit((x + 1) % L, y, z), spin_bit(x, (y + 1) % L, z), spin_bit(x, y, (z + 1) % L)};
    for (int d = 0; d < 3; ++d) {
      // J S_i S_j = -1 (unsatisfied, energy +1) iff an odd number of the three bits is set
      E += ((s ^ nb[d] ^ abi_j(jabi, JW, d, i)) & 1) ? 1 : -1;
    }
  }
  const int64_t g = ri.walker_off + wl;
  ws.E[g] = E;
  ws.E_min[g] = E;
  ws.rt_state[g] = 0;
  ws.new_min[g] = 0;
  ws.rt_count[g] = 0;
  ws.t_first[g] = 0;
  ws.t_last[g] = 0;
}

// Per-realization integer sums over walkers (Sec. III bookkeeping): one block per realization.
__global__ void k_reduce_real(const RealInfo* __restrict__ reals, WalkerState ws, RealStatsDev* __restrict__ out) {
  const RealInfo ri = reals[blockIdx.x];
  uint64_t cnt = 0, time = 0;
  int emin = 0x7fffffff, nm = 0, with = 0;
  for (int wl = threadIdx.x; wl < ri.walkers; wl += blockDim.x) {
    const int64_t g = ri.walker_off + wl;
    const uint64_t c = ws.rt_count[g];
    cnt += c;
    if (c > 0) {
      time += ws.t_last[g] - ws.t_first[g];
      with += 1;
    }
    emin = min(emin, ws.E_min[g]);
    nm |= ws.new_min[g];
  }
  __shared__ uint64_t s_cnt[256], s_time[256];
  __shared__ int s_emin[256], s_nm[256], s_with[256];
  s_cnt[threadIdx.x] = cnt;
  s_time[threadIdx.x] = time;
  s_emin[threadIdx.x] = emin;
  s_nm[threadIdx.x] = nm;
  s_with[threadIdx.x] = with;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      s_cnt[threadIdx.x] += s_cnt[threadIdx.x + s];
      s_time[threadIdx.x] += s_time[threadIdx.x + s];
      s_emin[threadIdx.x] = min(s_emin[threadIdx.x], s_emin[threadIdx.x + s]);
      s_nm[threadIdx.x] |= s_nm[threadIdx.x + s];
      s_with[threadIdx.x] += s_with[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    RealStatsDev o;
    o.rt_count = s_cnt[0];
    o.rt_time = s_time[0];
    o.E_min = s_emin[0];
    o.new_min = s_nm[0];
    o.walkers_with_trips = s_with[0];
    o.pad = 0;
    o.reserved = 0;
    out[blockIdx.x] = o;
  }
}

// ---------------------------------------------------------------------------------------------
// Host launchers.
hipError_t launch_gen_couplings(const RealInfo* reals, int n_real, uint32_t* jabi, uint64_t seed, hipStream_t s) {
  hipLaunchKernelGGL(k_gen_couplings, dim3(n_real), dim3(64), 0, s, reals, jabi, (uint32_t)seed,
                     (uint32_t)(seed >> 32));
  return hipGetLastError();
}

hipError_t launch_pack_couplings(RealInfo* reals, int n_real, const uint32_t* jabi, uint32_t* jk, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_couplings, dim3(n_real), dim3(256), 0, s, reals, jabi, jk);
  return hipGetLastError();
}

hipError_t launch_gen_spins(const RealInfo* reals, int r0, int nr, int max_walkers, uint32_t* spins, uint64_t seed,
                            hipStream_t s) {
  dim3 grid((max_walkers + 63) / 64, nr);
  hipLaunchKernelGGL(k_gen_spins, grid, dim3(64), 0, s, reals, r0, nr, spins, (uint32_t)seed, (uint32_t)(seed >> 32));
  return hipGetLastError();
}

hipError_t launch_pack_spins(const RealInfo* reals, int r, int wl0, int count, const int8_t* src, uint32_t* spins,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_pack_spins, dim3((count + 63) / 64), dim3(64), 0, s, reals, r, wl0, count, src, spins);
  return hipGetLastError();
}

hipError_t launch_unpack_spins(const RealInfo* reals, int r, int wl0, int count, const uint32_t* spins, int8_t* dst,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_unpack_spins, dim3((count + 63) / 64), dim3(64), 0, s, reals, r, wl0, count, spins, dst);
  return hipGetLastError();
}

hipError_t launch_energy(const RealInfo* reals, int n_real, int max_walkers, const uint32_t* jabi,
                         const uint32_t* spins, WalkerState ws, hipStream_t s) {
  dim3 grid((max_walkers + 63) / 64, n_real);
  hipLaunchKernelGGL(k_energy, grid, dim3(64), 0, s, reals, jabi, spins, ws);
  return hipGetLastError();
}

hipError_t launch_reduce_real(const RealInfo* reals, int n_real, WalkerState ws, RealStatsDev* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_real, dim3(n_real), dim3(256), 0, s, reals, ws, out);
  return hipGetLastError();
}

// Stuck-walker watch: a walker is flagged when its last completed round trip (without one: the
// clearing of its round-trip state, at sweep `since`) lies `window` or more sweeps before the
// sweep counter `now`. Stamps count attempts (sweep t, attempt a: t N + a + 1), so the age in
// whole sweeps is floor((now N - last) / N). One block per realization; flags (optional) per
// walker, the number flagged added to *count.
__global__ void k_stuck(const RealInfo* __restrict__ reals, WalkerState ws, uint64_t now, uint64_t since,
                        uint64_t window, uint8_t* __restrict__ flags, uint32_t* __restrict__ count) {
  const RealInfo ri = reals[blockIdx.x];
  const uint64_t N = (uint64_t)ri.N;
  const uint64_t end = now * N;
  uint32_t n = 0;
  for (int wl = threadIdx.x; wl < ri.walkers; wl += blockDim.x) {
    const int64_t g = ri.walker_off + wl;
    const uint64_t last = ws.rt_count[g] > 0 ? ws.t_last[g] : since * N;
    const uint64_t age = last < end ? (end - last) / N : 0;
    const bool stuck = age >= window;
    if (flags) flags[g] = stuck ? 1 : 0;
    n += stuck ? 1u : 0u;
  }
  if (n) atomicAdd(count, n);
}

hipError_t launch_stuck(const RealInfo* reals, int n_real, WalkerState ws, uint64_t now, uint64_t since,
                        uint64_t window, uint8_t* flags, uint32_t* count, hipStream_t s) {
  hipLaunchKernelGGL(k_stuck, dim3(n_real), dim3(256), 0, s, reals, ws, now, since, window, flags, count);
  return hipGetLastError();
}

// Round-trip times (Sec. III): tau_i = (sum of completed-trip time) / (number of trips) / N in
// sweeps, censored (NaN) below min_trips trips; tau_pop = mean of the uncensored tau_i. One block;
// the sum runs as a fixed-shape tree, so the result does not depend on scheduling.
__global__ void k_rt_stats(const RealInfo* __restrict__ reals, const RealStatsDev* __restrict__ st, int r0, int count,
                           uint64_t min_trips, double* __restrict__ tau, RtSummaryDev* __restrict__ out) {
  __shared__ double s_sum[256];
  __shared__ uint64_t s_trips[256];
  __shared__ int s_used[256];
  double sum = 0.0;
  uint64_t trips = 0;
  int used = 0;
  for (int i = threadIdx.x; i < count; i += blockDim.x) {
    const int r = r0 + i;
    const RealStatsDev d = st[r];
    trips += d.rt_count;
    double ti = __builtin_nan("");
    if (d.rt_count >= min_trips && d.rt_count > 0) {
      ti = (double)d.rt_time / (double)d.rt_count / (double)reals[r].N;
      sum += ti;
      used += 1;
    }
    tau[i] = ti;
  }
  s_sum[threadIdx.x] = sum;
  s_trips[threadIdx.x] = trips;
  s_used[threadIdx.x] = used;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      s_sum[threadIdx.x] += s_sum[threadIdx.x + s];
      s_trips[threadIdx.x] += s_trips[threadIdx.x + s];
      s_used[threadIdx.x] += s_used[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    RtSummaryDev o;
    o.tau_pop = s_used[0] > 0 ? s_sum[0] / (double)s_used[0] : __builtin_nan("");
    o.trips = s_trips[0];
    o.n_used = s_used[0];
    o.n_censored = count - s_used[0];
    *out = o;
  }
}

hipError_t launch_rt_stats(const RealInfo* reals, const RealStatsDev* stats, int r0, int count, uint64_t min_trips,
                           double* tau, RtSummaryDev* out, hipStream_t s) {
  hipLaunchKernelGGL(k_rt_stats, dim3(1), dim3(256), 0, s, reals, stats, r0, count, min_trips, tau, out);
  return hipGetLastError();
}

}  // namespace nfm
