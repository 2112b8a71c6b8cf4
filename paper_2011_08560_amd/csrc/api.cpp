// C ABI of libnfm (include/nfm.h): context, workspace layout, argument checking and
// kernel launches on the caller's stream. All device memory is the caller's workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <fstream>
#include <map>
#include <sstream>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/nfm.h"
#include "kernels.hpp"

using nfm::RealInfo;

namespace {

constexpr size_t kAlign = 256;
constexpr uint32_t kMaxSweepsPerLaunch = 1024;
constexpr int kNoBottom = -(1 << 20);  // far below any energy; keeps (k - row0) * 32 in int range

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  size_t reals, waves, jabi, jk, spins, ws_i32, ws_u64, tables, hist, lnw, klo, ktop, trace, rstats, staging, total;
  size_t recs, rec_f64, rec_vis;
  size_t pt_slot, pt_acc, pt_metro, pt_swap, pt_q, rt_tau, rt_sum, wl_f64, wl_hst, wl_info;
  size_t order, counter, snap_spins, snap_i32, snap_u64, snap_hist;
  int32_t pt_dcap;            // exchange-table width capacity: max over the batch of 3N/2 + 1
  int64_t total_walkers, total_waves, levels_total, jabi_words, jk_words, spin_words, table_words;
  size_t staging_bytes;
};

bool valid_L(int L) { return nfm::sweep_supported(L); }

// Deterministic workspace layout of a batch (the same for nfm_workspace_bytes and nfm_create).
bool make_layout(const nfm_batch_desc* d, Layout* lay, std::string* why) {
  if (!d || d->n_real < 1 || !d->L || !d->walkers) {
    *why = "batch description needs n_real >= 1 and L/walkers arrays";
    return false;
  }
  if (d->trace_capacity < 0) {
    *why = "trace_capacity must be >= 0";
    return false;
  }
  Layout l{};
  size_t max_stage = 0;
  for (int r = 0; r < d->n_real; ++r) {
    const int L = d->L[r], W = d->walkers[r];
    if (!valid_L(L)) {
      *why = "unsupported L (even, 2..12): realization " + std::to_string(r);
      return false;
    }
    if (W < 64 || W % 64 != 0) {
      *why = "walkers per realization must be a positive multiple of 64: realization " + std::to_string(r);
      return false;
    }
    const int N = L * L * L;
    l.total_walkers += W;
    l.total_waves += W / 64;
    l.levels_total += nfm::level_capacity(N);
    l.jabi_words += 3 * nfm::abi_plane_words(N);
    l.jk_words += nfm::jk_words(L);
    l.spin_words += (int64_t)W * nfm::walker_words(L);
    l.table_words += (int64_t)nfm::level_capacity(N) * 8;
    max_stage = std::max(max_stage, (size_t)W * N);
    l.pt_dcap = std::max<int32_t>(l.pt_dcap, 3 * N / 2 + 1);
  }
  max_stage = std::max(max_stage, (size_t)l.jabi_words * 4);
  l.staging_bytes = max_stage;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + std::max<size_t>(bytes, 1));
    return o;
  };
  l.reals = take(sizeof(RealInfo) * d->n_real);
  l.waves = take(sizeof(int32_t) * 2 * l.total_waves);
  l.jabi = take(4 * (size_t)l.jabi_words);
  l.jk = take(4 * (size_t)l.jk_words);
  l.spins = take(4 * (size_t)l.spin_words);
  l.ws_i32 = take(4 * 4 * (size_t)l.total_walkers);
  l.ws_u64 = take(8 * 3 * (size_t)l.total_walkers);
  l.tables = take(4 * (size_t)l.table_words);
  l.hist = take(8 * (size_t)l.levels_total);
  l.lnw = take(8 * (size_t)l.levels_total);
  l.klo = take(4 * (size_t)d->n_real);
  l.ktop = take(4 * (size_t)d->n_real);
  l.trace = take(4 * (size_t)l.total_walkers * (size_t)d->trace_capacity);
  l.rstats = take(sizeof(nfm::RealStatsDev) * d->n_real);
  l.staging = take(l.staging_bytes);
  l.recs = take(sizeof(nfm::RecInfo) * d->n_real);
  l.rec_f64 = take(8 * 5 * (size_t)l.levels_total);
  l.rec_vis = take((size_t)l.levels_total);
  l.pt_slot = take(4 * (size_t)l.total_walkers);
  l.pt_acc = take(8 * (size_t)l.total_walkers);
  l.pt_metro = take(4 * 8 * (size_t)nfm::kMaxReplicas * (size_t)d->n_real);
  l.pt_swap = take(4 * (size_t)(nfm::kMaxReplicas - 1) * (size_t)l.pt_dcap);
  l.pt_q = take(8 * (size_t)nfm::kMaxReplicas * (size_t)d->n_real);
  l.wl_f64 = take(8 * 2 * (size_t)l.levels_total);
  l.wl_hst = take(8 * (size_t)l.levels_total);
  l.wl_info = take(sizeof(nfm::WlInfo) * (size_t)d->n_real);
  l.rt_tau = take(8 * (size_t)d->n_real);
  l.rt_sum = take(sizeof(nfm::RtSummaryDev));
  l.order = take(4 * (size_t)l.total_waves);
  l.counter = take(256);
  l.snap_spins = take(4 * (size_t)l.spin_words);
  l.snap_i32 = take(4 * 4 * (size_t)l.total_walkers);
  l.snap_u64 = take(8 * 3 * (size_t)l.total_walkers);
  l.snap_hist = take(8 * (size_t)l.levels_total);
  l.total = off;
  *lay = l;
  return true;
}

}  // namespace

struct nfm_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  Layout lay{};
  int n_real = 0;
  uint64_t disorder_seed = 0, walker_seed = 0;
  int trace_cap = 0;                       // sweeps traced per walker of the traced range
  int64_t trace_slots = 0;                 // int32 entries of the workspace's trace region
  int64_t trace_w0 = 0, trace_nw = 0;      // traced walkers [trace_w0, trace_w0 + trace_nw)
  uint64_t sweeps = 0, trace_t0 = 0;
  bool couplings = false;
  int speculate = -1;                      // -1 auto, 0 off, 1 on
  int hist_mode = 0;                       // on-chip histogram: 0 auto, 1 window, 2 every level, 3 rows
  int ws_mode = 0;                         // generator wave: 0 auto, 1 never, 2 always
  uint32_t sweeps_per_launch = kMaxSweepsPerLaunch;
  int schedule = 0;                        // 0: one launch per lattice size, 1: persistent work queue
  int waves_per_cu = 0;                    // persistent grid: workgroups per CU (0 = as many as fit)
  int n_cu = 256;
  std::vector<RealInfo> reals;
  // waves grouped by L
  std::vector<int> group_L;
  std::vector<int64_t> group_first_wave, group_n_waves;
  // split persistent launch (schedule 2): the second stream, and the fork / join events between
  // it and the context's stream
  hipStream_t split_stream = nullptr;
  hipEvent_t split_fork = nullptr, split_join = nullptr;
  std::string err;

  RealInfo* d_reals() { return (RealInfo*)(ws + lay.reals); }
  int32_t* d_waves() { return (int32_t*)(ws + lay.waves); }
  uint32_t* d_jabi() { return (uint32_t*)(ws + lay.jabi); }
  uint32_t* d_jk() { return (uint32_t*)(ws + lay.jk); }
  uint32_t* d_spins() { return (uint32_t*)(ws + lay.spins); }
  uint32_t* d_tables() { return (uint32_t*)(ws + lay.tables); }
  unsigned long long* d_hist() { return (unsigned long long*)(ws + lay.hist); }
  double* d_lnw() { return (double*)(ws + lay.lnw); }
  int32_t* d_klo() { return (int32_t*)(ws + lay.klo); }
  int32_t* d_ktop() { return (int32_t*)(ws + lay.ktop); }
  int32_t* d_trace() { return (int32_t*)(ws + lay.trace); }
  nfm::RealStatsDev* d_rstats() { return (nfm::RealStatsDev*)(ws + lay.rstats); }
  void* d_staging() { return ws + lay.staging; }
  nfm::RecInfo* d_recs() { return (nfm::RecInfo*)(ws + lay.recs); }
  nfm::RecArrays rec_arrays() {
    nfm::RecArrays a;
    double* f = (double*)(ws + lay.rec_f64);
    const int64_t n = lay.levels_total;
    a.b = f;
    a.p = f + n;
    a.S = f + 2 * n;
    a.lnP = f + 3 * n;
    a.lnW = f + 4 * n;
    a.visited = (unsigned char*)(ws + lay.rec_vis);
    return a;
  }
  bool rec_ready = false;
  int pt_M = 0;                            // parallel tempering: slots per set
  std::vector<double> pt_T;                // per realization kMaxReplicas temperatures (slot order)
  uint64_t pt_t_reset = 0;                 // sweep counter when the exchange counters were cleared
  uint64_t rt_reset = 0;                   // sweep counter when the round-trip state was last cleared
  int32_t* d_pt_slot() { return (int32_t*)(ws + lay.pt_slot); }
  uint64_t* d_pt_acc() { return (uint64_t*)(ws + lay.pt_acc); }
  uint32_t* d_pt_metro() { return (uint32_t*)(ws + lay.pt_metro); }
  double* d_pt_q() { return (double*)(ws + lay.pt_q); }
  nfm::WlArrays wl_arrays() {
    double* f = (double*)(ws + lay.wl_f64);
    return nfm::WlArrays{f, (unsigned long long*)(ws + lay.wl_hst), f + lay.levels_total};
  }
  nfm::WlInfo* d_wl_info() { return (nfm::WlInfo*)(ws + lay.wl_info); }
  bool wl_ready = false;
  uint32_t* d_pt_swap() { return (uint32_t*)(ws + lay.pt_swap); }
  nfm::WalkerState walker_state() {
    nfm::WalkerState s;
    const int64_t W = lay.total_walkers;
    int32_t* i32 = (int32_t*)(ws + lay.ws_i32);
    uint64_t* u64 = (uint64_t*)(ws + lay.ws_u64);
    s.E = i32;
    s.E_min = i32 + W;
    s.rt_state = i32 + 2 * W;
    s.new_min = i32 + 3 * W;
    s.rt_count = u64;
    s.t_first = u64 + W;
    s.t_last = u64 + 2 * W;
    return s;
  }
};

namespace {

nfm_status fail(nfm_ctx* c, nfm_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

#define NFM_HIP(c, call)                                                                   \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess) return fail((c), NFM_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define NFM_GUARD(c)                                   \
  if (!(c)) return NFM_EINVAL;                         \
  if (hipSetDevice((c)->device) != hipSuccess) return fail((c), NFM_EDEVICE, "hipSetDevice failed")

#define NFM_TRY(c, ...)                                                          \
  try {                                                                          \
    __VA_ARGS__                                                                  \
  } catch (const std::bad_alloc&) {                                              \
    return fail((c), NFM_EDEVICE, "host allocation failed");                     \
  } catch (...) {                                                                \
    return fail((c), NFM_EDEVICE, "unexpected host exception");                  \
  }

nfm_status push_reals(nfm_ctx* c) {
  NFM_HIP(c, hipMemcpyAsync(c->d_reals(), c->reals.data(), sizeof(RealInfo) * c->n_real, hipMemcpyHostToDevice,
                            c->stream));
  NFM_HIP(c, hipStreamSynchronize(c->stream));
  return NFM_OK;
}

nfm_status pull_reals(nfm_ctx* c) {
  NFM_HIP(c, hipMemcpyAsync(c->reals.data(), c->d_reals(), sizeof(RealInfo) * c->n_real, hipMemcpyDeviceToHost,
                            c->stream));
  NFM_HIP(c, hipStreamSynchronize(c->stream));
  return NFM_OK;
}

int max_walkers(const nfm_ctx* c) {
  int m = 0;
  for (const auto& r : c->reals) m = std::max(m, r.walkers);
  return m;
}

// realization owning global walker index w
int real_of_walker(const nfm_ctx* c, int64_t w) {
  for (int r = 0; r < c->n_real; ++r)
    if (w >= c->reals[r].walker_off && w < c->reals[r].walker_off + c->reals[r].walkers) return r;
  return -1;
}

}  // namespace

extern "C" {

nfm_status nfm_workspace_bytes(const nfm_batch_desc* desc, size_t* bytes) {
  if (!bytes) return NFM_EINVAL;
  Layout l;
  std::string why;
  if (!make_layout(desc, &l, &why)) return NFM_EINVAL;
  *bytes = l.total;
  return NFM_OK;
}

nfm_status nfm_create(nfm_ctx** out, const nfm_batch_desc* desc, void* dev_workspace, size_t workspace_bytes,
                      int device, void* hip_stream) {
  if (!out) return NFM_EINVAL;
  *out = nullptr;
  Layout l;
  std::string why;
  if (!make_layout(desc, &l, &why)) return NFM_EINVAL;
  if (!dev_workspace || ((uintptr_t)dev_workspace % kAlign) != 0) return NFM_EINVAL;
  if (workspace_bytes < l.total) return NFM_ESIZE;
  nfm_ctx* c = new (std::nothrow) nfm_ctx();
  if (!c) return NFM_EDEVICE;
  try {
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->ws = (char*)dev_workspace;
    c->lay = l;
    c->n_real = desc->n_real;
    c->disorder_seed = desc->disorder_seed;
    c->walker_seed = desc->walker_seed;
    c->trace_cap = desc->trace_capacity;
    c->trace_slots = l.total_walkers * (int64_t)desc->trace_capacity;
    c->trace_w0 = 0;
    c->trace_nw = l.total_walkers;
    c->reals.resize(desc->n_real);
    int64_t woff = 0, soff = 0, loff = 0, toff = 0, jaoff = 0, jkoff = 0;
    for (int r = 0; r < desc->n_real; ++r) {
      RealInfo& ri = c->reals[r];
      std::memset(&ri, 0, sizeof(ri));
      ri.L = desc->L[r];
      ri.N = ri.L * ri.L * ri.L;
      ri.e_base = -3 * ri.N;
      ri.K = nfm::level_capacity(ri.N);
      ri.walkers = desc->walkers[r];
      ri.row0 = 0;
      ri.rows = 0;
      ri.e_bot = kNoBottom;
      ri.e_top = 0;
      ri.real_id = desc->first_real_id + (uint32_t)r;
      ri.walker_off = woff;
      ri.spin_off = soff;
      ri.level_off = loff;
      ri.table_off = toff;
      ri.jabi_off = jaoff;
      ri.jk_off = jkoff;
      woff += ri.walkers;
      soff += (int64_t)ri.walkers * nfm::walker_words(ri.L);
      loff += nfm::level_capacity(ri.N);
      toff += (int64_t)nfm::level_capacity(ri.N) * 8;
      jaoff += 3 * nfm::abi_plane_words(ri.N);
      jkoff += nfm::jk_words(ri.L);
    }
    // waves grouped by L (ascending), in realization order within a group
    std::vector<int32_t> waves;
    for (int L = 2; L <= nfm::kMaxL; L += 2) {
      const int64_t first = (int64_t)waves.size() / 2;
      for (int r = 0; r < desc->n_real; ++r) {
        if (c->reals[r].L != L) continue;
        for (int wl = 0; wl < c->reals[r].walkers; wl += 64) {
          waves.push_back(r);
          waves.push_back(wl);
        }
      }
      const int64_t n = (int64_t)waves.size() / 2 - first;
      if (n > 0) {
        c->group_L.push_back(L);
        c->group_first_wave.push_back(first);
        c->group_n_waves.push_back(n);
      }
    }
    // device arrays: wave_real[total_waves] then wave_wl[total_waves]
    std::vector<int32_t> wr(l.total_waves), wwl(l.total_waves);
    for (int64_t i = 0; i < l.total_waves; ++i) {
      wr[i] = waves[2 * i];
      wwl[i] = waves[2 * i + 1];
    }
    if (hipSetDevice(device) != hipSuccess) {
      delete c;
      return NFM_EDEVICE;
    }
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0)
      c->n_cu = ncu;
    nfm_status st = NFM_OK;
    // work-queue order: longest items (largest N) first, realization order within a size
    std::vector<int32_t> order(l.total_waves);
    for (int64_t i = 0; i < l.total_waves; ++i) order[i] = (int32_t)i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
      return c->reals[wr[a]].N > c->reals[wr[b]].N;
    });
    if (hipMemcpyAsync(c->ws + l.order, order.data(), 4 * order.size(), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipMemcpyAsync(c->d_waves(), wr.data(), 4 * wr.size(), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipMemcpyAsync(c->d_waves() + l.total_waves, wwl.data(), 4 * wwl.size(), hipMemcpyHostToDevice,
                       c->stream) != hipSuccess ||
        hipMemsetAsync(c->ws + l.ws_i32, 0, 4 * 4 * (size_t)l.total_walkers, c->stream) != hipSuccess ||
        hipMemsetAsync(c->ws + l.ws_u64, 0, 8 * 3 * (size_t)l.total_walkers, c->stream) != hipSuccess ||
        hipMemsetAsync(c->ws + l.hist, 0, 8 * (size_t)l.levels_total, c->stream) != hipSuccess ||
        hipMemsetAsync(c->ws + l.spins, 0, 4 * (size_t)l.spin_words, c->stream) != hipSuccess)
      st = NFM_EDEVICE;
    if (st == NFM_OK) st = push_reals(c);
    if (st != NFM_OK) {
      delete c;
      return st;
    }
  } catch (...) {
    delete c;
    return NFM_EDEVICE;
  }
  *out = c;
  return NFM_OK;
}

static void drop_split_stream(nfm_ctx* c) {
  if (c->split_stream) {
    (void)hipStreamSynchronize(c->split_stream);
    (void)hipStreamDestroy(c->split_stream);
  }
  if (c->split_fork) (void)hipEventDestroy(c->split_fork);
  if (c->split_join) (void)hipEventDestroy(c->split_join);
  c->split_stream = nullptr;
  c->split_fork = c->split_join = nullptr;
}

void nfm_destroy(nfm_ctx* ctx) {
  if (!ctx) return;
  if (hipSetDevice(ctx->device) == hipSuccess) {
    (void)hipStreamSynchronize(ctx->stream);
    drop_split_stream(ctx);
  }
  delete ctx;
}

const char* nfm_last_error(const nfm_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int32_t nfm_n_real(const nfm_ctx* c) { return c ? c->n_real : 0; }
int64_t nfm_n_walkers(const nfm_ctx* c) { return c ? c->lay.total_walkers : 0; }
int32_t nfm_levels(const nfm_ctx* c, int32_t r) { return (c && r >= 0 && r < c->n_real) ? c->reals[r].K : 0; }
int32_t nfm_e_base(const nfm_ctx* c, int32_t r) { return (c && r >= 0 && r < c->n_real) ? c->reals[r].e_base : 0; }
int64_t nfm_level_offset(const nfm_ctx* c, int32_t r) {
  return (c && r >= 0 && r < c->n_real) ? c->reals[r].level_off : -1;
}
int64_t nfm_levels_total(const nfm_ctx* c) { return c ? c->lay.levels_total : 0; }
int64_t nfm_walker_offset(const nfm_ctx* c, int32_t r) {
  return (c && r >= 0 && r < c->n_real) ? c->reals[r].walker_off : -1;
}
uint64_t nfm_sweep_counter(const nfm_ctx* c) { return c ? c->sweeps : 0; }

static nfm_status after_couplings(nfm_ctx* c) {
  hipError_t e = nfm::launch_pack_couplings(c->d_reals(), c->n_real, c->d_jabi(), c->d_jk(), c->stream);
  if (e != hipSuccess) return fail(c, NFM_EDEVICE, std::string("pack_couplings: ") + hipGetErrorString(e));
  nfm_status s = pull_reals(c);
  if (s != NFM_OK) return s;
  for (auto& r : c->reals) {  // tables refer to the old level set
    r.row0 = 0;
    r.rows = 0;
  }
  c->couplings = true;
  return push_reals(c);
}

nfm_status nfm_init_couplings(nfm_ctx* c) {
  NFM_GUARD(c);
  NFM_TRY(c, {
    hipError_t e = nfm::launch_gen_couplings(c->d_reals(), c->n_real, c->d_jabi(), c->disorder_seed, c->stream);
    if (e != hipSuccess) return fail(c, NFM_EDEVICE, std::string("gen_couplings: ") + hipGetErrorString(e));
    return after_couplings(c);
  })
}

nfm_status nfm_set_couplings(nfm_ctx* c, int32_t r0, int32_t count, const uint32_t* host_words) {
  NFM_GUARD(c);
  if (!host_words || r0 < 0 || count < 1 || r0 + count > c->n_real)
    return fail(c, NFM_EINVAL, "set_couplings: bad realization range or null pointer");
  NFM_TRY(c, {
    const int64_t first = c->reals[r0].jabi_off;
    const int64_t last = c->reals[r0 + count - 1].jabi_off + 3 * nfm::abi_plane_words(c->reals[r0 + count - 1].N);
    NFM_HIP(c, hipMemcpyAsync(c->d_jabi() + first, host_words, 4 * (size_t)(last - first), hipMemcpyHostToDevice,
                              c->stream));
    return after_couplings(c);
  })
}

nfm_status nfm_get_couplings(nfm_ctx* c, int32_t r0, int32_t count, uint32_t* host_words) {
  NFM_GUARD(c);
  if (!host_words || r0 < 0 || count < 1 || r0 + count > c->n_real)
    return fail(c, NFM_EINVAL, "get_couplings: bad realization range or null pointer");
  const int64_t first = c->reals[r0].jabi_off;
  const int64_t last = c->reals[r0 + count - 1].jabi_off + 3 * nfm::abi_plane_words(c->reals[r0 + count - 1].N);
  NFM_HIP(c, hipMemcpyAsync(host_words, c->d_jabi() + first, 4 * (size_t)(last - first), hipMemcpyDeviceToHost,
                            c->stream));
  NFM_HIP(c, hipStreamSynchronize(c->stream));
  return NFM_OK;
}

nfm_status nfm_init_spins(nfm_ctx* c) {
  NFM_GUARD(c);
  hipError_t e = nfm::launch_gen_spins(c->d_reals(), 0, c->n_real, max_walkers(c), c->d_spins(), c->walker_seed,
                                       c->stream);
  if (e != hipSuccess) return fail(c, NFM_EDEVICE, std::string("gen_spins: ") + hipGetErrorString(e));
  return NFM_OK;
}

static nfm_status spins_io(nfm_ctx* c, int64_t w0, int64_t count, const int8_t* src, int8_t* dst) {
  if ((!src && !dst) || w0 < 0 || count < 1 || w0 + count > c->lay.total_walkers)
    return fail(c, NFM_EINVAL, "spins: bad walker range or null pointer");
  NFM_TRY(c, {
    int64_t w = w0, done = 0;
    size_t host_off = 0;  // walkers of different realizations may have different N
    while (done < count) {
      const int r = real_of_walker(c, w);
      const RealInfo& ri = c->reals[r];
      const int64_t wl0 = w - ri.walker_off;
      const int64_t n = std::min<int64_t>(count - done, ri.walkers - wl0);
      const size_t bytes = (size_t)n * ri.N;
      int8_t* stage = (int8_t*)c->d_staging();
      if (src) {
        NFM_HIP(c, hipMemcpyAsync(stage, src + host_off, bytes, hipMemcpyHostToDevice, c->stream));
        hipError_t e = nfm::launch_pack_spins(c->d_reals(), r, (int)wl0, (int)n, stage, c->d_spins(), c->stream);
        if (e != hipSuccess) return fail(c, NFM_EDEVICE, std::string("pack_spins: ") + hipGetErrorString(e));
        NFM_HIP(c, hipStreamSynchronize(c->stream));
      } else {
        hipError_t e = nfm::launch_unpack_spins(c->d_reals(), r, (int)wl0, (int)n, c->d_spins(), stage, c->stream);
        if (e != hipSuccess) return fail(c, NFM_EDEVICE, std::string("unpack_spins: ") + hipGetErrorString(e));
        NFM_HIP(c, hipMemcpyAsync(dst + host_off, stage, bytes, hipMemcpyDeviceToHost, c->stream));
        NFM_HIP(c, hipStreamSynchronize(c->stream));
      }
      done += n;
      w += n;
      host_off += bytes;
    }
    return NFM_OK;
  })
}

nfm_status nfm_set_spins(nfm_ctx* c, int64_t w0, int64_t count, const int8_t* host_spins) {
  NFM_GUARD(c);
  if (!host_spins) return fail(c, NFM_EINVAL, "set_spins: null pointer");
  return spins_io(c, w0, count, host_spins, nullptr);
}

nfm_status nfm_get_spins(nfm_ctx* c, int64_t w0, int64_t count, int8_t* host_spins) {
  NFM_GUARD(c);
  if (!host_spins) return fail(c, NFM_EINVAL, "get_spins: null pointer");
  return spins_io(c, w0, count, nullptr, host_spins);
}

nfm_status nfm_compute_energies(nfm_ctx* c) {
  NFM_GUARD(c);
  if (!c->couplings) return fail(c, NFM_ESTATE, "compute_energies: couplings not set");
  hipError_t e = nfm::launch_energy(c->d_reals(), c->n_real, max_walkers(c), c->d_jabi(), c->d_spins(),
                                    c->walker_state(), c->stream);
  if (e != hipSuccess) return fail(c, NFM_EDEVICE, std::string("energy: ") + hipGetErrorString(e));
  c->rt_reset = c->sweeps;
  return NFM_OK;
}

nfm_status nfm_set_thresholds(nfm_ctx* c, int32_t r, const uint32_t* host_thr, int32_t row0, int32_t rows) {
  NFM_GUARD(c);
  if (!c->couplings) return fail(c, NFM_ESTATE, "set_thresholds: couplings not set");
  if (!host_thr || r < 0 || r >= c->n_real) return fail(c, NFM_EINVAL, "set_thresholds: bad realization");
  RealInfo& ri = c->reals[r];
  if (rows < 1 || row0 < 0 || row0 + rows > ri.K) return fail(c, NFM_EINVAL, "set_thresholds: rows outside [0, K)");
  NFM_HIP(c, hipMemcpyAsync(c->d_tables() + ri.table_off, host_thr, 4 * 8 * (size_t)rows, hipMemcpyHostToDevice,
                            c->stream));
  ri.row0 = row0;
  ri.rows = rows;
  return push_reals(c);
}

nfm_status nfm_get_thresholds(nfm_ctx* c, int32_t r, uint32_t* host_thr, int32_t* row0, int32_t* rows) {
  NFM_GUARD(c);
  if (r < 0 || r >= c->n_real || !row0 || !rows) return fail(c, NFM_EINVAL, "get_thresholds: bad arguments");
  const RealInfo& ri = c->reals[r];
  *row0 = ri.row0;
  *rows = ri.rows;
  if (host_thr && ri.rows > 0) {
    NFM_HIP(c, hipMemcpyAsync(host_thr, c->d_tables() + ri.table_off, 4 * 8 * (size_t)ri.rows, hipMemcpyDeviceToHost,
                              c->stream));
    NFM_HIP(c, hipStreamSynchronize(c->stream));
  }
  return NFM_OK;
}

nfm_status nfm_set_weights_lnw(nfm_ctx* c, const double* host_lnw, const int32_t* k_lo, const int32_t* k_top) {
  NFM_GUARD(c);
  if (!c->couplings) return fail(c, NFM_ESTATE, "set_weights_lnw: couplings not set");
  if (!host_lnw || !k_lo || !k_top) return fail(c, NFM_EINVAL, "set_weights_lnw: null pointer");
  for (int r = 0; r < c->n_real; ++r)
    if (k_lo[r] < 0 || k_top[r] >= c->reals[r].K || k_lo[r] > k_top[r])
      return fail(c, NFM_EINVAL, "set_weights_lnw: need 0 <= k_lo <= k_top < K, realization " + std::to_string(r));
  NFM_HIP(c, hipMemcpyAsync(c->d_lnw(), host_lnw, 8 * (size_t)c->lay.levels_total, hipMemcpyHostToDevice, c->stream));
  NFM_HIP(c, hipMemcpyAsync(c->d_klo(), k_lo, 4 * (size_t)c->n_real, hipMemcpyHostToDevice, c->stream));
  NFM_HIP(c, hipMemcpyAsync(c->d_ktop(), k_top, 4 * (size_t)c->n_real, hipMemcpyHostToDevice, c->stream));
  hipError_t e = nfm::launch_build_tables(c->d_reals(), c->n_real, c->d_lnw(), c->d_klo(), c->d_ktop(),
                                          c->d_tables(), c->stream);
  if (e != hipSuccess) return fail(c, NFM_EDEVICE, std::string("build_tables: ") + hipGetErrorString(e));
  return pull_reals(c);
}

nfm_status nfm_set_rt_bounds(nfm_ctx* c, int32_t r, int32_t e_bot, int32_t e_top) {
  NFM_GUARD(c);
  if (r < 0 || r >= c->n_real) return fail(c, NFM_EINVAL, "set_rt_bounds: bad realization");
  const int N = c->reals[r].N;
  if (e_bot < -4 * N || e_bot > 4 * N || e_top < -4 * N || e_top > 4 * N)
    return fail(c, NFM_EINVAL, "set_rt_bounds: bounds outside [-4N, 4N]");
  c->reals[r].e_bot = e_bot;
  c->reals[r].e_top = e_top;
  return push_reals(c);
}

static nfm::SweepArgs muca_args(nfm_ctx* c, uint64_t t0, uint32_t n, int trace_cap) {
  nfm::SweepArgs a{};
  a.reals = c->d_reals();
  a.wave_real = c->d_waves();
  a.wave_wl = c->d_waves() + c->lay.total_waves;
  a.spins = c->d_spins();
  a.jk = c->d_jk();
  a.tables = c->d_tables();
  a.ws = c->walker_state();
  a.hist = c->d_hist();
  a.trace = c->d_trace();
  a.trace_cap = trace_cap;
  a.trace_t0 = c->trace_t0;
  a.trace_w0 = c->trace_w0;
  a.trace_nw = c->trace_nw;
  a.t0 = t0;
  a.n_sweeps = n;
  a.walker_seed = c->walker_seed;
  return a;
}

// The split persistent launch (schedule 2). A sweep of the whole batch is bound by the serial
// chains of its largest lattices (one attempt after another per walker, Sec. II). Their waves run
// as a persistent queue of their own in the SIMD-exclusive kernel form, each alone on a SIMD and so
// at the chain's own issue rate, beside a second persistent queue over the remaining sizes (in the
// form compiled for them) on the SIMDs left free. The second queue is launched on its own stream
// behind a short wait, so that the first one is placed first.
struct SplitPart {
  int64_t first = 0, n = 0;   // slice of the work-queue order
  int maxl = 0, lds_rows = 1, K = 1;
};

static bool plan_split(const nfm_ctx* c, SplitPart* big, SplitPart* rest) {
  const int G = (int)c->group_L.size();   // sizes ascending; the order lists waves longest first
  if (G < 2) return false;
  *big = SplitPart{};
  *rest = SplitPart{};
  big->n = c->group_n_waves[G - 1];
  big->maxl = c->group_L[G - 1];
  rest->first = big->n;
  rest->n = c->lay.total_waves - big->n;
  rest->maxl = c->group_L[G - 2];
  for (const auto& ri : c->reals) {
    SplitPart* p = ri.L == big->maxl ? big : rest;
    p->lds_rows = std::max(p->lds_rows, ri.rows);
    p->K = std::max(p->K, ri.K);
  }
  return rest->n > 0;
}

static bool ensure_split_stream(nfm_ctx* c) {
  if (c->split_stream) return true;
  if (hipStreamCreateWithFlags(&c->split_stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->split_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->split_join, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    c->err = "split launch unavailable: stream or event creation failed";
    drop_split_stream(c);
    return false;
  }
  return true;
}

// Launch n multicanonical sweeps starting at sweep t0 under the given tuning (no checks).
static nfm_status muca_launches(nfm_ctx* c, uint64_t t0, uint64_t n_sweeps, int speculate, uint32_t per_launch,
                                int schedule, int waves_per_cu, int hist_mode, int ws_mode, int trace_cap) {
  int lds_all = 1, k_all = 1;
  for (const auto& ri : c->reals) {
    lds_all = std::max(lds_all, ri.rows);
    k_all = std::max(k_all, ri.K);
  }
  // schedule 2 splits off the largest size (a batch of one size runs as the plain persistent queue)
  SplitPart big, rest;
  const bool split = schedule == 2 && plan_split(c, &big, &rest) && ensure_split_stream(c);
  uint64_t done = 0;
  while (done < n_sweeps) {
    const uint32_t chunk = (uint32_t)std::min<uint64_t>(per_launch, n_sweeps - done);
    nfm::SweepArgs a = muca_args(c, t0 + done, chunk, trace_cap);
    if (split) {
      const bool spec = speculate == 1;
      const int32_t* order = (const int32_t*)(c->ws + c->lay.order);
      uint32_t* counter = (uint32_t*)(c->ws + c->lay.counter);
      // at most half the SIMDs go to the largest lattices; the rest of the queue over the SIMDs left
      const int64_t simds = 4LL * c->n_cu;
      const int64_t grid_big = std::max<int64_t>(1, std::min<int64_t>(big.n, simds / 2));
      // the other sizes: as many workgroups as fit on the whole device (those that find no room
      // beside the largest lattices' waves start when a slot frees and take what the queue has left)
      const int per_cu = std::max(1, nfm::queue_blocks_per_cu(spec, rest.lds_rows, rest.K, hist_mode, rest.maxl));
      const int64_t grid_rest = std::max<int64_t>(1, std::min<int64_t>(rest.n, (int64_t)per_cu * c->n_cu));
      NFM_HIP(c, hipEventRecord(c->split_fork, c->stream));
      hipError_t e = nfm::launch_muca_queue(a, order, (int)big.n, counter, (int)grid_big, c->n_cu, big.lds_rows, big.K,
                                            hist_mode, spec, c->stream, big.maxl, true);
      if (e != hipSuccess) return fail(c, NFM_EDEVICE, std::string("muca_queue (largest): ") + hipGetErrorString(e));
      NFM_HIP(c, hipStreamWaitEvent(c->split_stream, c->split_fork, 0));
      e = nfm::launch_hold(c->split_stream);
      if (e == hipSuccess)
        e = nfm::launch_muca_queue(a, order + rest.first, (int)rest.n, counter + 16, (int)grid_rest, c->n_cu,
                                   rest.lds_rows, rest.K, hist_mode, spec, c->split_stream, rest.maxl, false);
      if (e != hipSuccess) return fail(c, NFM_EDEVICE, std::string("muca_queue (rest): ") + hipGetErrorString(e));
      NFM_HIP(c, hipEventRecord(c->split_join, c->split_stream));
      NFM_HIP(c, hipStreamWaitEvent(c->stream, c->split_join, 0));
      nfm::note_partitioned_launch(spec);
    } else if (schedule >= 1) {
      const bool spec = speculate == 1;
      const int maxl = c->group_L.empty() ? nfm::kMaxL : c->group_L.back();
      int wpc = schedule == 1 ? waves_per_cu : 0;
      if (wpc <= 0) wpc = std::max(1, nfm::queue_blocks_per_cu(spec, lds_all, k_all, hist_mode, maxl));
      const int64_t grid = std::min<int64_t>(c->lay.total_waves, (int64_t)wpc * c->n_cu);
      hipError_t e = nfm::launch_muca_queue(a, (const int32_t*)(c->ws + c->lay.order), (int)c->lay.total_waves,
                                            (uint32_t*)(c->ws + c->lay.counter), (int)grid, c->n_cu, lds_all, k_all,
                                            hist_mode, spec, c->stream, maxl);
      if (e != hipSuccess) return fail(c, NFM_EDEVICE, std::string("muca_queue: ") + hipGetErrorString(e));
    } else {
      for (size_t g = 0; g < c->group_L.size(); ++g) {
        const int L = c->group_L[g];
        int lds_rows = 1, hist_levels = 1;
        for (const auto& ri : c->reals)
          if (ri.L == L) {
            lds_rows = std::max(lds_rows, ri.rows);
            hist_levels = std::max(hist_levels, ri.K);
          }
        a.wave_real = c->d_waves() + c->group_first_wave[g];
        a.wave_wl = c->d_waves() + c->lay.total_waves + c->group_first_wave[g];
        // Speculation is off unless asked for: the table read of the plain form is already
        // overlapped with generator work, which costs fewer instructions than a second read.
        const bool spec = speculate == 1;
        hipError_t e = nfm::launch_muca_sweeps(L, a, (int)c->group_n_waves[g], lds_rows, hist_levels, c->n_cu,
                                                     hist_mode, ws_mode, spec, c->stream);
        if (e != hipSuccess) return fail(c, NFM_EDEVICE, std::string("muca_sweeps: ") + hipGetErrorString(e));
      }
    }
    done += chunk;
  }
  return NFM_OK;
}

nfm_status nfm_run_sweeps(nfm_ctx* c, uint64_t n_sweeps) {
  NFM_GUARD(c);
  if (!c->couplings) return fail(c, NFM_ESTATE, "run_sweeps: couplings not set");
  for (int r = 0; r < c->n_real; ++r)
    if (c->reals[r].rows < 1) return fail(c, NFM_ESTATE, "run_sweeps: no threshold table, realization " + std::to_string(r));
  if (n_sweeps > (uint64_t)UINT32_MAX - c->sweeps)   // written so that it cannot wrap
    return fail(c, NFM_ERANGE, "run_sweeps: the sweep counter must stay below 2^32");
  nfm_status st = muca_launches(c, c->sweeps, n_sweeps, c->speculate, c->sweeps_per_launch, c->schedule,
                                c->waves_per_cu, c->hist_mode, c->ws_mode, c->trace_cap);
  if (st != NFM_OK) return st;
  c->sweeps += n_sweeps;
  return NFM_OK;
}

nfm_status nfm_read_histograms(nfm_ctx* c, uint64_t* host_dst, int reset) {
  NFM_GUARD(c);
  if (!host_dst) return fail(c, NFM_EINVAL, "read_histograms: null pointer");
  NFM_HIP(c, hipMemcpyAsync(host_dst, c->d_hist(), 8 * (size_t)c->lay.levels_total, hipMemcpyDeviceToHost, c->stream));
  if (reset) NFM_HIP(c, hipMemsetAsync(c->d_hist(), 0, 8 * (size_t)c->lay.levels_total, c->stream));
  NFM_HIP(c, hipStreamSynchronize(c->stream));
  return NFM_OK;
}

nfm_status nfm_reset_histograms(nfm_ctx* c) {
  NFM_GUARD(c);
  NFM_HIP(c, hipMemsetAsync(c->d_hist(), 0, 8 * (size_t)c->lay.levels_total, c->stream));
  return NFM_OK;
}

nfm_status nfm_read_walkers(nfm_ctx* c, nfm_walker_stats* host_dst) {
  NFM_GUARD(c);
  if (!host_dst) return fail(c, NFM_EINVAL, "read_walkers: null pointer");
  NFM_TRY(c, {
    const int64_t W = c->lay.total_walkers;
    std::vector<int32_t> i32(4 * W);
    std::vector<uint64_t> u64(3 * W);
    NFM_HIP(c, hipMemcpyAsync(i32.data(), c->ws + c->lay.ws_i32, 4 * i32.size(), hipMemcpyDeviceToHost, c->stream));
    NFM_HIP(c, hipMemcpyAsync(u64.data(), c->ws + c->lay.ws_u64, 8 * u64.size(), hipMemcpyDeviceToHost, c->stream));
    NFM_HIP(c, hipStreamSynchronize(c->stream));
    for (int64_t w = 0; w < W; ++w) {
      host_dst[w].E = i32[w];
      host_dst[w].E_min = i32[W + w];
      host_dst[w].rt_state = i32[2 * W + w];
      host_dst[w].new_min = i32[3 * W + w];
      host_dst[w].rt_count = u64[w];
      host_dst[w].t_first = u64[W + w];
      host_dst[w].t_last = u64[2 * W + w];
    }
    return NFM_OK;
  })
}

nfm_status nfm_read_realizations(nfm_ctx* c, nfm_real_stats* host_dst) {
  NFM_GUARD(c);
  if (!host_dst) return fail(c, NFM_EINVAL, "read_realizations: null pointer");
  static_assert(sizeof(nfm_real_stats) == sizeof(nfm::RealStatsDev), "layout");
  hipError_t e = nfm::launch_reduce_real(c->d_reals(), c->n_real, c->walker_state(), c->d_rstats(), c->stream);
  if (e != hipSuccess) return fail(c, NFM_EDEVICE, std::string("reduce_real: ") + hipGetErrorString(e));
  NFM_HIP(c, hipMemcpyAsync(host_dst, c->d_rstats(), sizeof(nfm_real_stats) * c->n_real, hipMemcpyDeviceToHost,
                            c->stream));
  NFM_HIP(c, hipStreamSynchronize(c->stream));
  return NFM_OK;
}

nfm_status nfm_read_trace(nfm_ctx* c, int32_t* host_dst, int32_t* n_valid) {
  NFM_GUARD(c);
  if (!n_valid) return fail(c, NFM_EINVAL, "read_trace: null pointer");
  const uint64_t done = c->sweeps - c->trace_t0;
  *n_valid = (int32_t)std::min<uint64_t>(done, (uint64_t)c->trace_cap);
  if (c->trace_cap > 0 && c->trace_nw > 0) {
    if (!host_dst) return fail(c, NFM_EINVAL, "read_trace: null pointer");
    NFM_HIP(c, hipMemcpyAsync(host_dst, c->d_trace(), 4 * (size_t)c->trace_nw * c->trace_cap,
                              hipMemcpyDeviceToHost, c->stream));
    NFM_HIP(c, hipStreamSynchronize(c->stream));
  }
  return NFM_OK;
}

nfm_status nfm_reset_trace(nfm_ctx* c) {
  NFM_GUARD(c);
  c->trace_t0 = c->sweeps;
  return NFM_OK;
}

nfm_status nfm_trace_range(const nfm_ctx* c, int64_t* walker_begin, int64_t* count, int32_t* capacity) {
  if (!c || !walker_begin || !count || !capacity) return NFM_EINVAL;
  *walker_begin = c->trace_w0;
  *count = c->trace_nw;
  *capacity = c->trace_cap;
  return NFM_OK;
}

nfm_status nfm_trace_config(nfm_ctx* c, int64_t walker_begin, int64_t count, int32_t capacity) {
  NFM_GUARD(c);
  if (walker_begin < 0 || count < 0 || capacity < 0 || walker_begin > c->lay.total_walkers ||
      count > c->lay.total_walkers - walker_begin)
    return fail(c, NFM_EINVAL, "trace_config: walkers [begin, begin + count) must lie in the batch, capacity >= 0");
  if (count > 0 && capacity > 0 && count > c->trace_slots / capacity)
    return fail(c, NFM_ESIZE, "trace_config: count x capacity exceeds the trace the workspace holds (" +
                                  std::to_string(c->trace_slots) + " entries)");
  c->trace_w0 = walker_begin;
  c->trace_nw = count;
  c->trace_cap = (count > 0) ? capacity : 0;
  c->trace_t0 = c->sweeps;
  return NFM_OK;
}

const char* nfm_last_kernel(const nfm_ctx* c) { return c ? nfm::last_sweep_kernel() : "none"; }

nfm_status nfm_sync(nfm_ctx* c) {
  NFM_GUARD(c);
  NFM_HIP(c, hipStreamSynchronize(c->stream));
  return NFM_OK;
}

// ---------------------------------------------------------------------------------------------
// Checkpoint / resume. Blob: header, the host scalars of the context, its tempering
// temperatures, then a byte copy of the whole device workspace (every device structure in it
// holds offsets, not addresses, so the copy is valid at any workspace address).
namespace {
constexpr char kCkptMagic[8] = {'N', 'F', 'M', 'C', 'K', 'P', 'T', '1'};
constexpr uint32_t kCkptVersion = 4;   // 4: the sweep of the last round-trip clearing is part of the header
struct CkptHeader {
  char magic[8];
  uint32_t version, n_real;
  uint64_t disorder_seed, walker_seed, batch_hash, workspace_bytes;
  int32_t trace_cap, couplings, speculate, hist_mode, ws_mode, pad;
  uint32_t sweeps_per_launch;
  int32_t schedule, waves_per_cu, rec_ready, pt_M, wl_ready;
  uint64_t sweeps, trace_t0, pt_t_reset;
  int64_t trace_slots, trace_w0, trace_nw;
  uint64_t rt_reset;
};

// FNV-1a over every realization's size, walker count and id: the layout of the workspace
uint64_t batch_hash(const nfm_ctx* c) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](int64_t v) {
    for (int i = 0; i < 8; ++i) {
      h ^= (uint64_t)((v >> (8 * i)) & 0xFF);
      h *= 1099511628211ull;
    }
  };
  for (const auto& r : c->reals) {
    mix(r.L);
    mix(r.walkers);
    mix(r.real_id);
  }
  return h;
}

size_t ckpt_bytes(const nfm_ctx* c) {
  return sizeof(CkptHeader) + sizeof(double) * (size_t)c->n_real * nfm::kMaxReplicas + c->lay.total;
}
}  // namespace

nfm_status nfm_checkpoint_bytes(const nfm_ctx* c, size_t* bytes) {
  if (!c || !bytes) return NFM_EINVAL;
  *bytes = ckpt_bytes(c);
  return NFM_OK;
}

nfm_status nfm_checkpoint(nfm_ctx* c, void* host_blob, size_t capacity) {
  NFM_GUARD(c);
  if (!host_blob) return fail(c, NFM_EINVAL, "checkpoint: null buffer");
  if (capacity < ckpt_bytes(c)) return fail(c, NFM_ESIZE, "checkpoint: buffer smaller than nfm_checkpoint_bytes()");
  CkptHeader h{};
  std::memcpy(h.magic, kCkptMagic, 8);
  h.version = kCkptVersion;
  h.n_real = (uint32_t)c->n_real;
  h.disorder_seed = c->disorder_seed;
  h.walker_seed = c->walker_seed;
  h.batch_hash = batch_hash(c);
  h.workspace_bytes = c->lay.total;
  h.trace_cap = c->trace_cap;
  h.couplings = c->couplings ? 1 : 0;
  h.speculate = c->speculate;
  h.hist_mode = c->hist_mode;
  h.ws_mode = c->ws_mode;
  h.sweeps_per_launch = c->sweeps_per_launch;
  h.schedule = c->schedule;
  h.waves_per_cu = c->waves_per_cu;
  h.rec_ready = c->rec_ready ? 1 : 0;
  h.pt_M = c->pt_M;
  h.wl_ready = c->wl_ready ? 1 : 0;
  h.sweeps = c->sweeps;
  h.trace_t0 = c->trace_t0;
  h.pt_t_reset = c->pt_t_reset;
  h.trace_slots = c->trace_slots;
  h.trace_w0 = c->trace_w0;
  h.trace_nw = c->trace_nw;
  h.rt_reset = c->rt_reset;
  char* out = (char*)host_blob;
  std::memcpy(out, &h, sizeof(h));
  double* T = (double*)(out + sizeof(h));
  const size_t nT = (size_t)c->n_real * nfm::kMaxReplicas;
  for (size_t i = 0; i < nT; ++i) T[i] = i < c->pt_T.size() ? c->pt_T[i] : 0.0;
  // everything queued on the stream so far is part of the state
  NFM_HIP(c, hipMemcpyAsync(out + sizeof(h) + sizeof(double) * nT, c->ws, c->lay.total, hipMemcpyDeviceToHost,
                            c->stream));
  NFM_HIP(c, hipStreamSynchronize(c->stream));
  return NFM_OK;
}

nfm_status nfm_restore(nfm_ctx* c, const void* host_blob, size_t size) {
  NFM_GUARD(c);
  if (!host_blob || size < sizeof(CkptHeader)) return fail(c, NFM_EINVAL, "restore: no checkpoint");
  CkptHeader h;
  std::memcpy(&h, host_blob, sizeof(h));
  if (std::memcmp(h.magic, kCkptMagic, 8) != 0 || h.version != kCkptVersion)
    return fail(c, NFM_EINVAL, "restore: not a checkpoint of this library version");
  if (h.n_real != (uint32_t)c->n_real || h.batch_hash != batch_hash(c) || h.workspace_bytes != c->lay.total ||
      h.disorder_seed != c->disorder_seed || h.walker_seed != c->walker_seed || h.trace_slots != c->trace_slots)
    return fail(c, NFM_EINVAL, "restore: checkpoint of a different batch (sizes, walkers, ids, seeds or trace)");
  if (size < ckpt_bytes(c)) return fail(c, NFM_ESIZE, "restore: checkpoint truncated");
  if (h.sweeps > (uint64_t)UINT32_MAX || h.trace_t0 > h.sweeps || h.pt_t_reset > h.sweeps || h.rt_reset > h.sweeps)
    return fail(c, NFM_EINVAL, "restore: sweep counters out of range");
  if (h.trace_w0 < 0 || h.trace_nw < 0 || h.trace_w0 + h.trace_nw > c->lay.total_walkers || h.trace_cap < 0 ||
      (h.trace_nw > 0 && h.trace_cap > 0 && h.trace_nw > h.trace_slots / h.trace_cap))
    return fail(c, NFM_EINVAL, "restore: traced walker range out of range");
  NFM_TRY(c, {
    const char* in = (const char*)host_blob;
    const size_t nT = (size_t)c->n_real * nfm::kMaxReplicas;
    NFM_HIP(c, hipMemcpyAsync(c->ws, in + sizeof(h) + sizeof(double) * nT, c->lay.total, hipMemcpyHostToDevice,
                              c->stream));
    NFM_HIP(c, hipStreamSynchronize(c->stream));
    const double* T = (const double*)(in + sizeof(h));
    c->pt_T.assign(T, T + nT);
    c->couplings = h.couplings != 0;
    c->speculate = h.speculate;
    c->hist_mode = h.hist_mode;
    c->ws_mode = h.ws_mode;
    c->sweeps_per_launch = h.sweeps_per_launch;
    c->schedule = h.schedule;
    c->waves_per_cu = h.waves_per_cu;
    c->rec_ready = h.rec_ready != 0;
    c->pt_M = h.pt_M;
    c->wl_ready = h.wl_ready != 0;
    c->sweeps = h.sweeps;
    c->trace_t0 = h.trace_t0;
    c->trace_cap = h.trace_cap;
    c->trace_w0 = h.trace_w0;
    c->trace_nw = h.trace_nw;
    c->pt_t_reset = h.pt_t_reset;
    c->rt_reset = h.rt_reset;
    return pull_reals(c);   // table rows, bounds and energies base as the checkpoint had them
  })
}


nfm_status nfm_set_histograms(nfm_ctx* c, const uint64_t* host_src) {
  NFM_GUARD(c);
  if (!host_src) return fail(c, NFM_EINVAL, "set_histograms: null pointer");
  NFM_HIP(c, hipMemcpyAsync(c->d_hist(), host_src, 8 * (size_t)c->lay.levels_total, hipMemcpyHostToDevice, c->stream));
  NFM_HIP(c, hipStreamSynchronize(c->stream));
  return NFM_OK;
}

nfm_status nfm_reset_round_trips(nfm_ctx* c) {
  NFM_GUARD(c);
  const int64_t W = c->lay.total_walkers;
  nfm::WalkerState ws = c->walker_state();
  NFM_HIP(c, hipMemsetAsync(ws.rt_state, 0, 4 * (size_t)W, c->stream));
  NFM_HIP(c, hipMemsetAsync(ws.new_min, 0, 4 * (size_t)W, c->stream));
  NFM_HIP(c, hipMemsetAsync(c->ws + c->lay.ws_u64, 0, 8 * 3 * (size_t)W, c->stream));
  c->rt_reset = c->sweeps;
  return NFM_OK;
}

nfm_status nfm_stuck_walkers(nfm_ctx* c, uint64_t window_sweeps, uint8_t* device_flags, int64_t* host_count) {
  NFM_GUARD(c);
  if (!host_count) return fail(c, NFM_EINVAL, "stuck_walkers: null count");
  // the count sits past the two work-queue counters of the persistent launches
  uint32_t* d_count = (uint32_t*)(c->ws + c->lay.counter) + 32;
  NFM_HIP(c, hipMemsetAsync(d_count, 0, 4, c->stream));
  hipError_t e = nfm::launch_stuck(c->d_reals(), c->n_real, c->walker_state(), c->sweeps, c->rt_reset, window_sweeps,
                                   device_flags, d_count, c->stream);
  if (e != hipSuccess) return fail(c, NFM_EDEVICE, std::string("stuck_walkers: ") + hipGetErrorString(e));
  uint32_t n = 0;
  NFM_HIP(c, hipMemcpyAsync(&n, d_count, 4, hipMemcpyDeviceToHost, c->stream));
  NFM_HIP(c, hipStreamSynchronize(c->stream));
  *host_count = (int64_t)n;
  return NFM_OK;
}

static bool valid_profile(int profile, double dE, double alpha) {
  if (profile < 0 || profile > 2) return false;
  if (profile == 1 && !(dE > 0.0 && alpha <= 0.0)) return false;
  return true;
}

nfm_status nfm_rec_init(nfm_ctx* c, int32_t profile, double pl_dE, double pl_alpha) {
  NFM_GUARD(c);
  if (!c->couplings) return fail(c, NFM_ESTATE, "rec_init: couplings not set");
  if (!valid_profile(profile, pl_dE, pl_alpha)) return fail(c, NFM_EINVAL, "rec_init: bad profile");
  hipError_t e = nfm::launch_rec_init(c->d_reals(), c->d_recs(), c->n_real, c->rec_arrays(), c->walker_state(), profile,
                                      pl_dE, pl_alpha, c->d_tables(), c->stream);
  if (e != hipSuccess) return fail(c, NFM_EDEVICE, std::string("rec_init: ") + hipGetErrorString(e));
  NFM_HIP(c, hipMemsetAsync(c->d_hist(), 0, 8 * (size_t)c->lay.levels_total, c->stream));
  c->rec_ready = true;
  return pull_reals(c);
}

nfm_status nfm_rec_update(nfm_ctx* c, double f_tol, nfm_rec_info* host_info) {
  NFM_GUARD(c);
  if (!c->rec_ready) return fail(c, NFM_ESTATE, "rec_update: call nfm_rec_init first");
  if (!(f_tol >= 0.0 && f_tol <= 1.0)) return fail(c, NFM_EINVAL, "rec_update: f_tol outside [0, 1]");
  hipError_t e = nfm::launch_rec_update(c->d_reals(), c->d_recs(), c->n_real, c->rec_arrays(), c->walker_state(),
                                        c->d_hist(), c->d_tables(), f_tol, c->stream);
  if (e != hipSuccess) return fail(c, NFM_EDEVICE, std::string("rec_update: ") + hipGetErrorString(e));
  nfm_status st = pull_reals(c);
  if (st != NFM_OK || !host_info) return st;
  static_assert(sizeof(nfm_rec_info) == sizeof(nfm::RecInfo), "layout");
  NFM_HIP(c, hipMemcpyAsync(host_info, c->d_recs(), sizeof(nfm_rec_info) * c->n_real, hipMemcpyDeviceToHost, c->stream));
  NFM_HIP(c, hipStreamSynchronize(c->stream));
  return NFM_OK;
}

nfm_status nfm_rec_production(nfm_ctx* c, int32_t profile, double pl_dE, double pl_alpha) {
  NFM_GUARD(c);
  if (!c->rec_ready) return fail(c, NFM_ESTATE, "rec_production: call nfm_rec_init first");
  if (!valid_profile(profile, pl_dE, pl_alpha)) return fail(c, NFM_EINVAL, "rec_production: bad profile");
  hipError_t e = nfm::launch_rec_production(c->d_reals(), c->d_recs(), c->n_real, c->rec_arrays(), c->d_tables(),
                                            profile, pl_dE, pl_alpha, c->stream);
  if (e != hipSuccess) return fail(c, NFM_EDEVICE, std::string("rec_production: ") + hipGetErrorString(e));
  NFM_HIP(c, hipMemsetAsync(c->d_hist(), 0, 8 * (size_t)c->lay.levels_total, c->stream));
  return pull_reals(c);
}

// ------------------------------------------------------------------------------------------
// Wang-Landau estimate (batched form; see wl.hip).

nfm_status nfm_wl_init(nfm_ctx* c, double ln_f0) {
  NFM_GUARD(c);
  if (!c->couplings) return fail(c, NFM_ESTATE, "wl_init: couplings not set");
  if (!(ln_f0 > 0.0) || !std::isfinite(ln_f0)) return fail(c, NFM_EINVAL, "wl_init: ln_f0 must be positive and finite");
  hipError_t e = nfm::launch_wl_init(c->d_reals(), c->n_real, c->wl_arrays(), c->d_wl_info(), ln_f0, c->d_tables(),
                                     c->stream);
  if (e != hipSuccess) return fail(c, NFM_EDEVICE, std::string("wl_init: ") + hipGetErrorString(e));
  NFM_HIP(c, hipMemsetAsync(c->d_hist(), 0, 8 * (size_t)c->lay.levels_total, c->stream));
  c->wl_ready = true;
  return pull_reals(c);
}

nfm_status nfm_wl_update(nfm_ctx* c, double flat_tol, double ln_f_final, nfm_wl_info* host_info) {
  NFM_GUARD(c);
  if (!c->wl_ready) return fail(c, NFM_ESTATE, "wl_update: call nfm_wl_init first");
  if (!(flat_tol >= 0.0 && flat_tol <= 1.0) || !(ln_f_final > 0.0))
    return fail(c, NFM_EINVAL, "wl_update: flat_tol in [0, 1] and ln_f_final > 0");
  hipError_t e = nfm::launch_wl_update(c->d_reals(), c->n_real, c->wl_arrays(), c->d_wl_info(), c->d_hist(), flat_tol,
                                       ln_f_final, c->d_tables(), c->stream);
  if (e != hipSuccess) return fail(c, NFM_EDEVICE, std::string("wl_update: ") + hipGetErrorString(e));
  nfm_status st = pull_reals(c);
  if (st != NFM_OK || !host_info) return st;
  static_assert(sizeof(nfm_wl_info) == sizeof(nfm::WlInfo), "layout");
  NFM_HIP(c, hipMemcpyAsync(host_info, c->d_wl_info(), sizeof(nfm_wl_info) * c->n_real, hipMemcpyDeviceToHost, c->stream));
  NFM_HIP(c, hipStreamSynchronize(c->stream));
  return NFM_OK;
}

nfm_status nfm_wl_get(nfm_ctx* c, int32_t r, double* host_lng, uint64_t* host_hst, nfm_wl_info* info) {
  NFM_GUARD(c);
  if (!c->wl_ready) return fail(c, NFM_ESTATE, "wl_get: call nfm_wl_init first");
  if (r < 0 || r >= c->n_real) return fail(c, NFM_EINVAL, "wl_get: bad realization");
  const int64_t off = c->reals[r].level_off;
  const size_t n = (size_t)nfm::level_capacity(c->reals[r].N);
  nfm::WlArrays a = c->wl_arrays();
  if (host_lng) NFM_HIP(c, hipMemcpyAsync(host_lng, a.lng + off, 8 * n, hipMemcpyDeviceToHost, c->stream));
  if (host_hst) NFM_HIP(c, hipMemcpyAsync(host_hst, a.hst + off, 8 * n, hipMemcpyDeviceToHost, c->stream));
  if (info) NFM_HIP(c, hipMemcpyAsync(info, c->d_wl_info() + r, sizeof(nfm_wl_info), hipMemcpyDeviceToHost, c->stream));
  NFM_HIP(c, hipStreamSynchronize(c->stream));
  return NFM_OK;
}

nfm_status nfm_wl_to_rec(nfm_ctx* c, int32_t profile, double pl_dE, double pl_alpha) {
  NFM_GUARD(c);
  if (!c->wl_ready) return fail(c, NFM_ESTATE, "wl_to_rec: call nfm_wl_init first");
  if (!valid_profile(profile, pl_dE, pl_alpha)) return fail(c, NFM_EINVAL, "wl_to_rec: bad profile");
  hipError_t e = nfm::launch_wl_to_rec(c->d_reals(), c->d_recs(), c->n_real, c->rec_arrays(), c->wl_arrays(),
                                       c->d_wl_info(), profile, pl_dE, pl_alpha, c->stream);
  if (e == hipSuccess)
    e = nfm::launch_rec_weights(c->d_reals(), c->d_recs(), c->n_real, c->rec_arrays(), c->d_tables(), 1, c->stream);
  if (e != hipSuccess) return fail(c, NFM_EDEVICE, std::string("wl_to_rec: ") + hipGetErrorString(e));
  NFM_HIP(c, hipMemsetAsync(c->d_hist(), 0, 8 * (size_t)c->lay.levels_total, c->stream));
  c->rec_ready = true;
  return pull_reals(c);
}

nfm_status nfm_rec_read_info(nfm_ctx* c, nfm_rec_info* host_info) {
  NFM_GUARD(c);
  if (!host_info) return fail(c, NFM_EINVAL, "rec_read_info: null pointer");
  NFM_HIP(c, hipMemcpyAsync(host_info, c->d_recs(), sizeof(nfm_rec_info) * c->n_real, hipMemcpyDeviceToHost, c->stream));
  NFM_HIP(c, hipStreamSynchronize(c->stream));
  return NFM_OK;
}

nfm_status nfm_rec_get_state(nfm_ctx* c, int32_t r, double* b, double* p, double* S, double* lnP, double* lnW,
                             uint8_t* visited, nfm_rec_info* info) {
  NFM_GUARD(c);
  if (r < 0 || r >= c->n_real) return fail(c, NFM_EINVAL, "rec_get_state: bad realization");
  const int64_t off = c->reals[r].level_off;
  const size_t n = (size_t)nfm::level_capacity(c->reals[r].N);
  nfm::RecArrays a = c->rec_arrays();
  double* src[5] = {a.b, a.p, a.S, a.lnP, a.lnW};
  double* dst[5] = {b, p, S, lnP, lnW};
  for (int i = 0; i < 5; ++i)
    if (dst[i]) NFM_HIP(c, hipMemcpyAsync(dst[i], src[i] + off, 8 * n, hipMemcpyDeviceToHost, c->stream));
  if (visited) NFM_HIP(c, hipMemcpyAsync(visited, a.visited + off, n, hipMemcpyDeviceToHost, c->stream));
  if (info) NFM_HIP(c, hipMemcpyAsync(info, c->d_recs() + r, sizeof(nfm_rec_info), hipMemcpyDeviceToHost, c->stream));
  NFM_HIP(c, hipStreamSynchronize(c->stream));
  return NFM_OK;
}

nfm_status nfm_rec_set_state(nfm_ctx* c, int32_t r, const double* b, const double* p, const double* lnP,
                             const double* lnW, const uint8_t* visited, const nfm_rec_info* info) {
  NFM_GUARD(c);
  if (!c->couplings) return fail(c, NFM_ESTATE, "rec_set_state: couplings not set");
  if (r < 0 || r >= c->n_real || !b || !p || !lnP || !lnW || !visited || !info)
    return fail(c, NFM_EINVAL, "rec_set_state: bad arguments");
  const RealInfo& ri = c->reals[r];
  if (info->k_lo < 0 || info->k_top >= ri.K || info->k_lo > info->k_top || !valid_profile(info->profile, info->pl_dE, info->pl_alpha) ||
      info->k_seed < -1 || info->k_seed >= info->k_top)
    return fail(c, NFM_EINVAL, "rec_set_state: bad level range or profile");
  const int64_t off = ri.level_off;
  const size_t n = (size_t)nfm::level_capacity(ri.N);
  nfm::RecArrays a = c->rec_arrays();
  NFM_HIP(c, hipMemcpyAsync(a.b + off, b, 8 * n, hipMemcpyHostToDevice, c->stream));
  NFM_HIP(c, hipMemcpyAsync(a.p + off, p, 8 * n, hipMemcpyHostToDevice, c->stream));
  NFM_HIP(c, hipMemcpyAsync(a.lnP + off, lnP, 8 * n, hipMemcpyHostToDevice, c->stream));
  NFM_HIP(c, hipMemcpyAsync(a.lnW + off, lnW, 8 * n, hipMemcpyHostToDevice, c->stream));
  NFM_HIP(c, hipMemcpyAsync(a.visited + off, visited, n, hipMemcpyHostToDevice, c->stream));
  NFM_HIP(c, hipMemcpyAsync(c->d_recs() + r, info, sizeof(nfm_rec_info), hipMemcpyHostToDevice, c->stream));
  NFM_HIP(c, hipStreamSynchronize(c->stream));
  c->rec_ready = true;
  return NFM_OK;
}


nfm_status nfm_set_tuning(nfm_ctx* c, const nfm_tuning* t) {
  if (!c || !t) return NFM_EINVAL;
  if (t->speculate < -1 || t->speculate > 1 || t->sweeps_per_launch < 0 || t->sweeps_per_launch > (1 << 20) ||
      t->schedule < 0 || t->schedule > 2 ||
      t->waves_per_cu < 0 || t->waves_per_cu > 64 || t->hist < 0 || t->hist > 3 || t->ws < 0 || t->ws > 2)
    return fail(c, NFM_EINVAL,
                "set_tuning: speculate in {-1,0,1}, sweeps_per_launch in [0, 2^20], schedule in {0,1,2}, waves_per_cu in "
                "[0,64], hist in {0,1,2,3}, ws in {0,1,2}");
  c->speculate = t->speculate;
  c->sweeps_per_launch = t->sweeps_per_launch == 0 ? kMaxSweepsPerLaunch : (uint32_t)t->sweeps_per_launch;
  c->schedule = t->schedule;
  c->waves_per_cu = t->waves_per_cu;
  c->hist_mode = t->hist;
  c->ws_mode = t->ws;
  return NFM_OK;
}

nfm_status nfm_get_tuning(const nfm_ctx* c, nfm_tuning* t) {
  if (!c || !t) return NFM_EINVAL;
  t->speculate = c->speculate;
  t->sweeps_per_launch = (int32_t)c->sweeps_per_launch;
  t->schedule = c->schedule;
  t->waves_per_cu = c->waves_per_cu;
  t->hist = c->hist_mode;
  t->ws = c->ws_mode;
  return NFM_OK;
}

// Key of the autotuning cache: device, CU count, and the batch's mix of (L, walkers).
static std::string tune_key(nfm_ctx* c) {
  hipDeviceProp_t prop;
  std::string dev = "unknown";
  if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) dev = prop.gcnArchName;
  for (auto& ch : dev)
    if (ch == ' ' || ch == '|') ch = '_';
  std::map<int, int64_t> mix;
  for (const auto& r : c->reals) mix[r.L] += r.walkers;
  std::string k = dev + ":" + std::to_string(c->n_cu);
  for (const auto& kv : mix) k += ":L" + std::to_string(kv.first) + "x" + std::to_string(kv.second);
  return k;
}

static std::map<std::string, nfm_tuning>& tune_cache() {
  static std::map<std::string, nfm_tuning> m;
  return m;
}

nfm_status nfm_autotune(nfm_ctx* c, int32_t calib_sweeps, const char* cache_path, nfm_tune_result* results,
                        int32_t max_results, int32_t* n_results, nfm_tuning* best) {
  NFM_GUARD(c);
  if (!c->couplings) return fail(c, NFM_ESTATE, "autotune: couplings not set");
  for (int r = 0; r < c->n_real; ++r)
    if (c->reals[r].rows < 1) return fail(c, NFM_ESTATE, "autotune: no threshold table, realization " + std::to_string(r));
  if (calib_sweeps < 1 || max_results < 0 || (max_results > 0 && !results))
    return fail(c, NFM_EINVAL, "autotune: calib_sweeps >= 1 and a results array of max_results entries");
  if ((uint64_t)calib_sweeps > (uint64_t)UINT32_MAX - c->sweeps)
    return fail(c, NFM_ERANGE, "autotune: the sweep counter must stay below 2^32");
  NFM_TRY(c, {
    const std::string key = tune_key(c);
    int found = 0;
    nfm_tuning hit{};
    auto it = tune_cache().find(key);
    if (it != tune_cache().end()) {
      hit = it->second;
      found = 1;
    } else if (cache_path) {
      std::ifstream f(cache_path);
      std::string line;
      while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string k;
        nfm_tuning t{};
        if ((is >> k >> t.speculate >> t.sweeps_per_launch >> t.schedule >> t.waves_per_cu >> t.hist >> t.ws) &&
            k == key) {
          hit = t;
          found = 1;
        }
      }
    }
    if (n_results) *n_results = 0;
    if (found) {
      tune_cache()[key] = hit;
      nfm_status st = nfm_set_tuning(c, &hit);
      if (st == NFM_OK && best) *best = hit;
      return st;
    }
    // Snapshot the state the sweeps change, time every candidate on the live batch, restore.
    const Layout& l = c->lay;
    NFM_HIP(c, hipMemcpyAsync(c->ws + l.snap_spins, c->ws + l.spins, 4 * (size_t)l.spin_words, hipMemcpyDeviceToDevice, c->stream));
    NFM_HIP(c, hipMemcpyAsync(c->ws + l.snap_i32, c->ws + l.ws_i32, 16 * (size_t)l.total_walkers, hipMemcpyDeviceToDevice, c->stream));
    NFM_HIP(c, hipMemcpyAsync(c->ws + l.snap_u64, c->ws + l.ws_u64, 24 * (size_t)l.total_walkers, hipMemcpyDeviceToDevice, c->stream));
    NFM_HIP(c, hipMemcpyAsync(c->ws + l.snap_hist, c->ws + l.hist, 8 * (size_t)l.levels_total, hipMemcpyDeviceToDevice, c->stream));
    std::vector<nfm_tuning> cand;
    const int chunks[] = {16, 64, 256, 1024};
    for (int spec = 0; spec <= 1; ++spec)
      for (int ch : chunks) {
        // per-size launches: with and without the generator wave (speculation has none)
        cand.push_back(nfm_tuning{spec, ch, 0, 0, 0, 1});
        if (!spec) cand.push_back(nfm_tuning{spec, ch, 0, 0, 0, 2});
        cand.push_back(nfm_tuning{spec, ch, 1, 0, 0, 0});
        for (int wpc : {4, 8})
          if ((int64_t)wpc * c->n_cu < l.total_waves) cand.push_back(nfm_tuning{spec, ch, 1, wpc, 0, 0});
        SplitPart big, rest;
        const bool split = plan_split(c, &big, &rest);
        if (split) cand.push_back(nfm_tuning{spec, ch, 2, 0, 0, 0});
        // the on-chip histogram as the window alone for the persistent forms. Every level is left
        // to the automatic choice, which is made again at each launch: the tables grow over the
        // weight iteration, and a histogram of every level fixed at calibration (small tables)
        // costs resident workgroups later (measured 6 % slower on the mixed batch).
        if (ch == 256) {
          cand.push_back(nfm_tuning{spec, ch, 1, 0, 1, 0});
          if (split) cand.push_back(nfm_tuning{spec, ch, 2, 0, 1, 0});
        }
      }
    hipEvent_t e0, e1;
    NFM_HIP(c, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
      (void)hipEventDestroy(e0);
      return fail(c, NFM_EDEVICE, "autotune: hipEventCreate failed");
    }
    double attempts = 0.0;
    for (const auto& r : c->reals) attempts += (double)r.walkers * r.N;
    attempts *= (double)calib_sweeps;
    nfm_tuning bt = cand[0];
    double best_rate = -1.0;
    int nres = 0;
    nfm_status st = NFM_OK;
    // one untimed warm-up pass so that first-launch costs do not favour later candidates
    st = muca_launches(c, c->sweeps, (uint64_t)std::min(calib_sweeps, 64), 0, kMaxSweepsPerLaunch, 0, 0, 0, 0, 0);
    for (size_t i = 0; i < cand.size() && st == NFM_OK; ++i) {
      const nfm_tuning& t = cand[i];
      if (hipEventRecord(e0, c->stream) != hipSuccess) { st = fail(c, NFM_EDEVICE, "autotune: event"); break; }
      st = muca_launches(c, c->sweeps, (uint64_t)calib_sweeps, t.speculate, (uint32_t)t.sweeps_per_launch, t.schedule,
                         t.waves_per_cu, t.hist, t.ws, 0);
      if (st != NFM_OK) break;
      float ms = 0.f;
      if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        st = fail(c, NFM_EDEVICE, "autotune: timing failed");
        break;
      }
      const double rate = attempts / (ms * 1e-3);
      if (nres < max_results) results[nres++] = nfm_tune_result{t, rate};
      if (rate > best_rate) {
        best_rate = rate;
        bt = t;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    NFM_HIP(c, hipMemcpyAsync(c->ws + l.spins, c->ws + l.snap_spins, 4 * (size_t)l.spin_words, hipMemcpyDeviceToDevice, c->stream));
    NFM_HIP(c, hipMemcpyAsync(c->ws + l.ws_i32, c->ws + l.snap_i32, 16 * (size_t)l.total_walkers, hipMemcpyDeviceToDevice, c->stream));
    NFM_HIP(c, hipMemcpyAsync(c->ws + l.ws_u64, c->ws + l.snap_u64, 24 * (size_t)l.total_walkers, hipMemcpyDeviceToDevice, c->stream));
    NFM_HIP(c, hipMemcpyAsync(c->ws + l.hist, c->ws + l.snap_hist, 8 * (size_t)l.levels_total, hipMemcpyDeviceToDevice, c->stream));
    NFM_HIP(c, hipStreamSynchronize(c->stream));
    if (st != NFM_OK) return st;
    if (n_results) *n_results = nres;
    tune_cache()[key] = bt;
    if (cache_path) {
      std::ofstream f(cache_path, std::ios::app);
      if (f) f << key << " " << bt.speculate << " " << bt.sweeps_per_launch << " " << bt.schedule << " " << bt.waves_per_cu
               << " " << bt.hist << " " << bt.ws << "\n";
    }
    if (best) *best = bt;
    return nfm_set_tuning(c, &bt);
  })
}

// ------------------------------------------------------------------------------------------
// Parallel tempering (Sec. II, Eq. (8)).

static bool pt_valid_M(int M) { return M >= 2 && M <= nfm::kMaxReplicas; }

static bool pt_valid_temps(int M, const double* T) {
  if (!T) return false;
  for (int s = 0; s < M; ++s)
    if (!(T[s] > 0.0 && std::isfinite(T[s])) || (s > 0 && !(T[s] > T[s - 1]))) return false;
  return true;
}

// Sets of the walkers (one wave = 64 walkers holds floor(64/M) sets of M lanes).
static int64_t pt_sets_of(const nfm_ctx* c, int r) { return (int64_t)(c->reals[r].walkers / 64) * (64 / c->pt_M); }
static int64_t pt_sets_total(const nfm_ctx* c) { return (c->lay.total_walkers / 64) * (64 / c->pt_M); }

static uint32_t pt_quantize(double x) { return x >= 1.0 ? 0xFFFFFFFFu : (uint32_t)std::floor(std::ldexp(x, 32)); }

// Every realization's Metropolis rows (u-order, pad 0; step m = 3 - u, x = exp(-(1/T)(4m))) and
// the q of each pair, exp(4 (1/T_{s+1} - 1/T_s)), from the host temperatures (FP64), uploaded.
static nfm_status pt_upload(nfm_ctx* c) {
  const int M = c->pt_M, R = c->n_real, X = nfm::kMaxReplicas;
  std::vector<uint32_t> metro((size_t)R * X * 8, 0u);
  std::vector<double> q((size_t)R * X, 0.0);
  for (int r = 0; r < R; ++r) {
    const double* T = &c->pt_T[(size_t)r * X];
    for (int s = 0; s < M; ++s) {
      const double beta = 1.0 / T[s];
      for (int u = 0; u <= 6; ++u) {
        const int m = 3 - u;
        metro[((size_t)r * X + s) * 8 + u] = m <= 0 ? 0xFFFFFFFFu : pt_quantize(std::exp(-beta * (double)(4 * m)));
      }
      if (s + 1 < M) q[(size_t)r * X + s] = std::exp(4.0 * (1.0 / T[s + 1] - 1.0 / T[s]));
    }
  }
  NFM_HIP(c, hipMemcpyAsync(c->d_pt_metro(), metro.data(), 4 * metro.size(), hipMemcpyHostToDevice, c->stream));
  NFM_HIP(c, hipMemcpyAsync(c->d_pt_q(), q.data(), 8 * q.size(), hipMemcpyHostToDevice, c->stream));
  NFM_HIP(c, hipStreamSynchronize(c->stream));
  return NFM_OK;
}

nfm_status nfm_pt_init(nfm_ctx* c, int32_t M, const double* host_temps) {
  NFM_GUARD(c);
  if (!c->couplings) return fail(c, NFM_ESTATE, "pt_init: couplings not set");
  if (!pt_valid_M(M)) return fail(c, NFM_EINVAL, "pt_init: M must lie in [2, 64]");
  if (!pt_valid_temps(M, host_temps))
    return fail(c, NFM_EINVAL, "pt_init: temperatures must be positive, finite and strictly increasing");
  NFM_TRY(c, {
    c->pt_T.assign((size_t)c->n_real * nfm::kMaxReplicas, 0.0);
    for (int r = 0; r < c->n_real; ++r)
      for (int s = 0; s < M; ++s) c->pt_T[(size_t)r * nfm::kMaxReplicas + s] = host_temps[s];
    // configuration c of each set starts at slot c; idle lanes of a wave sit at slot 0
    const int spw = 64 / M;
    std::vector<int32_t> slot(c->lay.total_walkers);
    for (int64_t w = 0; w < c->lay.total_walkers; ++w) {   // walker offsets are multiples of 64
      const int lane = (int)(w % 64);
      slot[w] = lane < spw * M ? lane % M : 0;
    }
    c->pt_M = M;
    nfm_status st = pt_upload(c);
    if (st != NFM_OK) return st;
    NFM_HIP(c, hipMemcpyAsync(c->d_pt_slot(), slot.data(), 4 * slot.size(), hipMemcpyHostToDevice, c->stream));
    NFM_HIP(c, hipMemsetAsync(c->d_pt_acc(), 0, 8 * (size_t)c->lay.total_walkers, c->stream));
    NFM_HIP(c, hipStreamSynchronize(c->stream));
    c->pt_t_reset = c->sweeps;
    return NFM_OK;
  })
}

nfm_status nfm_pt_set_temps(nfm_ctx* c, int32_t r, const double* host_temps) {
  NFM_GUARD(c);
  if (c->pt_M == 0) return fail(c, NFM_ESTATE, "pt_set_temps: call nfm_pt_init first");
  if (r < 0 || r >= c->n_real) return fail(c, NFM_EINVAL, "pt_set_temps: bad realization");
  if (!pt_valid_temps(c->pt_M, host_temps))
    return fail(c, NFM_EINVAL, "pt_set_temps: temperatures must be positive, finite and strictly increasing");
  for (int s = 0; s < c->pt_M; ++s) c->pt_T[(size_t)r * nfm::kMaxReplicas + s] = host_temps[s];
  NFM_TRY(c, { return pt_upload(c); })
}

nfm_status nfm_pt_get_temps(nfm_ctx* c, int32_t r, double* host_temps) {
  NFM_GUARD(c);
  if (c->pt_M == 0) return fail(c, NFM_ESTATE, "pt_get_temps: call nfm_pt_init first");
  if (r < 0 || r >= c->n_real || !host_temps) return fail(c, NFM_EINVAL, "pt_get_temps: bad arguments");
  for (int s = 0; s < c->pt_M; ++s) host_temps[s] = c->pt_T[(size_t)r * nfm::kMaxReplicas + s];
  return NFM_OK;
}

nfm_status nfm_pt_get_tables(nfm_ctx* c, int32_t r, uint32_t* host_metro, uint32_t* host_swap, int32_t* M, int32_t* D) {
  NFM_GUARD(c);
  if (!M || !D) return fail(c, NFM_EINVAL, "pt_get_tables: null pointer");
  *M = c->pt_M;
  *D = 0;
  if (c->pt_M == 0) return NFM_OK;
  if (r < 0 || r >= c->n_real) return fail(c, NFM_EINVAL, "pt_get_tables: bad realization");
  NFM_TRY(c, {
    const int Mv = c->pt_M, cap = c->lay.pt_dcap;
    hipError_t e = nfm::launch_pt_swap_table(c->d_pt_q(), r, Mv, cap, c->d_pt_swap(), c->stream);
    if (e != hipSuccess) return fail(c, NFM_EDEVICE, std::string("pt_swap_table: ") + hipGetErrorString(e));
    std::vector<uint32_t> sw((size_t)(Mv - 1) * cap);
    NFM_HIP(c, hipMemcpyAsync(sw.data(), c->d_pt_swap(), 4 * sw.size(), hipMemcpyDeviceToHost, c->stream));
    if (host_metro)
      NFM_HIP(c, hipMemcpyAsync(host_metro, c->d_pt_metro() + (size_t)r * nfm::kMaxReplicas * 8,
                                4 * 8 * (size_t)Mv, hipMemcpyDeviceToHost, c->stream));
    NFM_HIP(c, hipStreamSynchronize(c->stream));
    int Dv = cap;
    for (int d = 1; d <= cap; ++d) {
      bool zero = true;
      for (int s = 0; s + 1 < Mv && zero; ++s) zero = sw[(size_t)s * cap + (d - 1)] == 0u;
      if (zero) {
        Dv = d;
        break;
      }
    }
    *D = Dv;
    if (host_swap)
      for (int s = 0; s + 1 < Mv; ++s)
        for (int d = 1; d <= Dv; ++d) host_swap[(size_t)s * Dv + (d - 1)] = sw[(size_t)s * cap + (d - 1)];
    return NFM_OK;
  })
}

nfm_status nfm_pt_adapt(nfm_ctx* c, double rate_lo, double rate_hi, double* host_rates, int32_t* n_outside) {
  NFM_GUARD(c);
  if (c->pt_M == 0) return fail(c, NFM_ESTATE, "pt_adapt: call nfm_pt_init first");
  if (!(rate_lo >= 0.0) || !(rate_hi <= 1.0) || !(rate_lo <= rate_hi))
    return fail(c, NFM_EINVAL, "pt_adapt: need 0 <= rate_lo <= rate_hi <= 1");
  const uint64_t t0 = c->pt_t_reset, t1 = c->sweeps;
  // sweeps t in [t0, t1) with t = s (mod 2): the exchange attempts of pair s per set
  const uint64_t n_even = (t1 + 1) / 2 - (t0 + 1) / 2, n_odd = t1 / 2 - t0 / 2;
  if (n_even == 0 || n_odd == 0) return fail(c, NFM_ESTATE, "pt_adapt: run at least two PT sweeps first");
  NFM_TRY(c, {
    const int M = c->pt_M;
    std::vector<uint64_t> acc((size_t)pt_sets_total(c) * (M - 1));
    NFM_HIP(c, hipMemcpyAsync(acc.data(), c->d_pt_acc(), 8 * acc.size(), hipMemcpyDeviceToHost, c->stream));
    NFM_HIP(c, hipStreamSynchronize(c->stream));
    int outside = 0;
    int64_t set0 = 0;
    std::vector<double> beta(M), rate(M - 1), gap(M - 1);
    for (int r = 0; r < c->n_real; ++r) {
      const int64_t ns = pt_sets_of(c, r);
      double* T = &c->pt_T[(size_t)r * nfm::kMaxReplicas];
      for (int s = 0; s < M; ++s) beta[s] = 1.0 / T[s];
      const double span = beta[0] - beta[M - 1];
      double total = 0.0;
      for (int s = 0; s + 1 < M; ++s) {
        uint64_t a = 0;
        for (int64_t g = 0; g < ns; ++g) a += acc[(size_t)(set0 + g) * (M - 1) + s];
        rate[s] = (double)a / ((double)ns * (double)((s % 2 == 0) ? n_even : n_odd));
        if (rate[s] < rate_lo || rate[s] > rate_hi) ++outside;
        if (host_rates) host_rates[(size_t)r * (M - 1) + s] = rate[s];
        // A = exp(-c gap^2) would be equalised by gap / sqrt(-ln A); half that step in log space,
        // at most a factor of 2 either way (near A = 1 -- neighbours sharing the ground state --
        // the Gaussian picture fails and the raw factor runs to 1000)
        const double a_c = std::min(std::max(rate[s], 1e-6), 1.0 - 1e-12);
        const double f = std::min(std::max(std::pow(-std::log(a_c), -0.25), 0.5), 2.0);
        gap[s] = (beta[s] - beta[s + 1]) * f;
        total += gap[s];
      }
      const double bmax = beta[M - 1];
      for (int s = 0; s + 2 < M; ++s) beta[s + 1] = beta[s] - gap[s] * (span / total);
      beta[M - 1] = bmax;   // both ends stay where they are
      for (int s = 0; s < M; ++s) T[s] = 1.0 / beta[s];
      set0 += ns;
    }
    if (n_outside) *n_outside = outside;
    nfm_status st = pt_upload(c);
    if (st != NFM_OK) return st;
    NFM_HIP(c, hipMemsetAsync(c->d_pt_acc(), 0, 8 * (size_t)c->lay.total_walkers, c->stream));
    NFM_HIP(c, hipStreamSynchronize(c->stream));
    c->pt_t_reset = c->sweeps;
    return NFM_OK;
  })
}

nfm_status nfm_pt_run_sweeps(nfm_ctx* c, uint64_t n_sweeps) {
  NFM_GUARD(c);
  if (c->pt_M == 0) return fail(c, NFM_ESTATE, "pt_run_sweeps: call nfm_pt_init first");
  if (n_sweeps > (uint64_t)UINT32_MAX - c->sweeps)   // written so that it cannot wrap
    return fail(c, NFM_ERANGE, "pt_run_sweeps: the sweep counter must stay below 2^32");
  uint64_t done = 0;
  while (done < n_sweeps) {
    const uint32_t chunk = (uint32_t)std::min<uint64_t>(c->sweeps_per_launch, n_sweeps - done);
    for (size_t g = 0; g < c->group_L.size(); ++g) {
      nfm::SweepArgs a{};
      a.reals = c->d_reals();
      a.wave_real = c->d_waves() + c->group_first_wave[g];
      a.wave_wl = c->d_waves() + c->lay.total_waves + c->group_first_wave[g];
      a.spins = c->d_spins();
      a.jk = c->d_jk();
      a.ws = c->walker_state();
      a.trace = c->d_trace();
      a.trace_cap = c->trace_cap;
      a.trace_t0 = c->trace_t0;
      a.trace_w0 = c->trace_w0;
      a.trace_nw = c->trace_nw;
      a.t0 = c->sweeps + done;
      a.n_sweeps = chunk;
      a.walker_seed = c->walker_seed;
      a.pt_metro = c->d_pt_metro();
      a.pt_q = c->d_pt_q();
      a.pt_slot = c->d_pt_slot();
      a.pt_acc = c->d_pt_acc();
      a.pt_M = c->pt_M;
      a.pt_spw = 64 / c->pt_M;
      a.pt_minv = (uint32_t)(0xFFFFFFFFu / (uint32_t)c->pt_M + 1u);   // ceil(2^32 / M): lane / M = mulhi(lane, minv)
      hipError_t e = nfm::launch_pt_sweeps(c->group_L[g], a, (int)c->group_n_waves[g], c->stream);
      if (e != hipSuccess) return fail(c, NFM_EDEVICE, std::string("pt_sweeps: ") + hipGetErrorString(e));
    }
    done += chunk;
  }
  c->sweeps += n_sweeps;
  return NFM_OK;
}

nfm_status nfm_pt_read_slots(nfm_ctx* c, int32_t* host_slots) {
  NFM_GUARD(c);
  if (c->pt_M == 0) return fail(c, NFM_ESTATE, "pt_read_slots: call nfm_pt_init first");
  if (!host_slots) return fail(c, NFM_EINVAL, "pt_read_slots: null pointer");
  NFM_HIP(c, hipMemcpyAsync(host_slots, c->d_pt_slot(), 4 * (size_t)c->lay.total_walkers, hipMemcpyDeviceToHost,
                            c->stream));
  NFM_HIP(c, hipStreamSynchronize(c->stream));
  return NFM_OK;
}

nfm_status nfm_pt_set_slots(nfm_ctx* c, const int32_t* host_slots) {
  NFM_GUARD(c);
  if (c->pt_M == 0) return fail(c, NFM_ESTATE, "pt_set_slots: call nfm_pt_init first");
  if (!host_slots) return fail(c, NFM_EINVAL, "pt_set_slots: null pointer");
  NFM_TRY(c, {
    const int M = c->pt_M;
    std::vector<char> seen(M);
    const int spw = 64 / M;
    for (int64_t w0 = 0; w0 < c->lay.total_walkers; w0 += 64) {
      for (int g = 0; g < spw; ++g) {
        std::fill(seen.begin(), seen.end(), 0);
        for (int k = 0; k < M; ++k) {
          const int32_t v = host_slots[w0 + g * M + k];
          if (v < 0 || v >= M || seen[v])
            return fail(c, NFM_EINVAL, "pt_set_slots: each set needs a permutation of 0..M-1");
          seen[v] = 1;
        }
      }
      for (int k = spw * M; k < 64; ++k)
        if (host_slots[w0 + k] != 0) return fail(c, NFM_EINVAL, "pt_set_slots: idle walkers stay at slot 0");
    }
    NFM_HIP(c, hipMemcpyAsync(c->d_pt_slot(), host_slots, 4 * (size_t)c->lay.total_walkers, hipMemcpyHostToDevice,
                              c->stream));
    NFM_HIP(c, hipStreamSynchronize(c->stream));
    return NFM_OK;
  })
}

nfm_status nfm_pt_read_exchanges(nfm_ctx* c, uint64_t* host_acc) {
  NFM_GUARD(c);
  if (c->pt_M == 0) return fail(c, NFM_ESTATE, "pt_read_exchanges: call nfm_pt_init first");
  if (!host_acc) return fail(c, NFM_EINVAL, "pt_read_exchanges: null pointer");
  const size_t n = (size_t)pt_sets_total(c) * (size_t)(c->pt_M - 1);
  NFM_HIP(c, hipMemcpyAsync(host_acc, c->d_pt_acc(), 8 * n, hipMemcpyDeviceToHost, c->stream));
  NFM_HIP(c, hipStreamSynchronize(c->stream));
  return NFM_OK;
}

// ------------------------------------------------------------------------------------------
// Round-trip statistics (Sec. III).

nfm_status nfm_rt_stats(nfm_ctx* c, int32_t r0, int32_t count, uint64_t min_trips, double* host_tau,
                        nfm_rt_summary* host_summary) {
  NFM_GUARD(c);
  if (r0 < 0 || count < 1 || r0 + count > c->n_real || !host_summary)
    return fail(c, NFM_EINVAL, "rt_stats: bad realization range or null pointer");
  static_assert(sizeof(nfm_rt_summary) == sizeof(nfm::RtSummaryDev), "layout");
  hipError_t e = nfm::launch_reduce_real(c->d_reals(), c->n_real, c->walker_state(), c->d_rstats(), c->stream);
  if (e != hipSuccess) return fail(c, NFM_EDEVICE, std::string("reduce_real: ") + hipGetErrorString(e));
  double* d_tau = (double*)(c->ws + c->lay.rt_tau);
  nfm::RtSummaryDev* d_sum = (nfm::RtSummaryDev*)(c->ws + c->lay.rt_sum);
  e = nfm::launch_rt_stats(c->d_reals(), c->d_rstats(), r0, count, min_trips, d_tau, d_sum, c->stream);
  if (e != hipSuccess) return fail(c, NFM_EDEVICE, std::string("rt_stats: ") + hipGetErrorString(e));
  if (host_tau) NFM_HIP(c, hipMemcpyAsync(host_tau, d_tau, 8 * (size_t)count, hipMemcpyDeviceToHost, c->stream));
  NFM_HIP(c, hipMemcpyAsync(host_summary, d_sum, sizeof(nfm_rt_summary), hipMemcpyDeviceToHost, c->stream));
  NFM_HIP(c, hipStreamSynchronize(c->stream));
  return NFM_OK;
}


// ------------------------------------------------------------------------------------------
// Learned seeding of the weight iteration.

nfm_status nfm_rec_seed(nfm_ctx* c, const double* host_b, const int32_t* host_k_seed) {
  NFM_GUARD(c);
  if (!c->rec_ready) return fail(c, NFM_ESTATE, "rec_seed: call nfm_rec_init first");
  if (!host_b || !host_k_seed) return fail(c, NFM_EINVAL, "rec_seed: null pointer");
  NFM_TRY(c, {
    std::vector<nfm_rec_info> info(c->n_real);
    NFM_HIP(c, hipMemcpyAsync(info.data(), c->d_recs(), sizeof(nfm_rec_info) * c->n_real, hipMemcpyDeviceToHost,
                              c->stream));
    NFM_HIP(c, hipStreamSynchronize(c->stream));
    for (int r = 0; r < c->n_real; ++r)
      if (host_k_seed[r] < -1 || host_k_seed[r] >= info[r].k_top)
        return fail(c, NFM_EINVAL, "rec_seed: k_seed must be -1 or in [0, k_top), realization " + std::to_string(r));
    // staging: the caller-weights region (levels_total doubles) and the k_lo region (n_real ints)
    NFM_HIP(c, hipMemcpyAsync(c->d_lnw(), host_b, 8 * (size_t)c->lay.levels_total, hipMemcpyHostToDevice, c->stream));
    NFM_HIP(c, hipMemcpyAsync(c->d_klo(), host_k_seed, 4 * (size_t)c->n_real, hipMemcpyHostToDevice, c->stream));
    hipError_t e = nfm::launch_rec_seed_copy(c->d_reals(), c->d_recs(), c->n_real, c->rec_arrays(), c->d_lnw(),
                                             c->d_klo(), c->stream);
    if (e != hipSuccess) return fail(c, NFM_EDEVICE, std::string("rec_seed: ") + hipGetErrorString(e));
    e = nfm::launch_rec_weights(c->d_reals(), c->d_recs(), c->n_real, c->rec_arrays(), c->d_tables(), 1, c->stream);
    if (e != hipSuccess) return fail(c, NFM_EDEVICE, std::string("rec_weights: ") + hipGetErrorString(e));
    return pull_reals(c);
  })
}

nfm_status nfm_rec_seed_grid(nfm_ctx* c, const float* dev_curves, int32_t* host_k_seed) {
  NFM_GUARD(c);
  if (!c->rec_ready) return fail(c, NFM_ESTATE, "rec_seed_grid: call nfm_rec_init first");
  if (!dev_curves) return fail(c, NFM_EINVAL, "rec_seed_grid: null pointer");
  hipError_t e = nfm::launch_rec_seed_grid(c->d_reals(), c->d_recs(), c->n_real, c->rec_arrays(), dev_curves,
                                           c->d_klo(), c->stream);
  if (e != hipSuccess) return fail(c, NFM_EDEVICE, std::string("rec_seed_grid: ") + hipGetErrorString(e));
  e = nfm::launch_rec_weights(c->d_reals(), c->d_recs(), c->n_real, c->rec_arrays(), c->d_tables(), 1, c->stream);
  if (e != hipSuccess) return fail(c, NFM_EDEVICE, std::string("rec_weights: ") + hipGetErrorString(e));
  if (host_k_seed)
    NFM_HIP(c, hipMemcpyAsync(host_k_seed, c->d_klo(), 4 * (size_t)c->n_real, hipMemcpyDeviceToHost, c->stream));
  return pull_reals(c);
}

nfm_status nfm_rec_targets(nfm_ctx* c, float* dev_y, float* dev_mask) {
  NFM_GUARD(c);
  if (!c->rec_ready) return fail(c, NFM_ESTATE, "rec_targets: call nfm_rec_init first");
  if (!dev_y || !dev_mask) return fail(c, NFM_EINVAL, "rec_targets: null pointer");
  hipError_t e = nfm::launch_rec_targets(c->d_reals(), c->d_recs(), c->n_real, c->rec_arrays(), dev_y, dev_mask,
                                         c->stream);
  if (e != hipSuccess) return fail(c, NFM_EDEVICE, std::string("rec_targets: ") + hipGetErrorString(e));
  return NFM_OK;
}

nfm_status nfm_set_canonical(nfm_ctx* c, double T) {
  NFM_GUARD(c);
  if (!c->couplings) return fail(c, NFM_ESTATE, "set_canonical: couplings not set");
  if (!(T > 0.0) || !std::isfinite(T)) return fail(c, NFM_EINVAL, "set_canonical: T must be positive and finite");
  hipError_t e = nfm::launch_canonical_tables(c->d_reals(), c->n_real, T, c->d_lnw(), c->d_klo(), c->d_ktop(),
                                              c->d_tables(), c->stream);
  if (e != hipSuccess) return fail(c, NFM_EDEVICE, std::string("canonical_tables: ") + hipGetErrorString(e));
  return pull_reals(c);
}

nfm_status nfm_features(nfm_ctx* c, float* dev_x) {
  NFM_GUARD(c);
  if (!c->couplings) return fail(c, NFM_ESTATE, "features: couplings not set");
  if (!dev_x) return fail(c, NFM_EINVAL, "features: null pointer");
  hipError_t e = nfm::launch_features(c->d_reals(), c->n_real, c->d_jabi(), c->d_hist(), dev_x, c->stream);
  if (e != hipSuccess) return fail(c, NFM_EDEVICE, std::string("features: ") + hipGetErrorString(e));
  return NFM_OK;
}

}  // extern "C"
