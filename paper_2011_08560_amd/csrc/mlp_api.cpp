// C ABI of the weight-seeding network (include/nfm.h, nfm_mlp_*): workspace layout, argument
// checks and the launch sequences of mlp.hip on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>
#include <string>

#include "../../include/nfm.h"
#include "mlp_internal.hpp"

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
int pad16(int b) { return (b + 15) / 16 * 16; }

struct MlpLayout {
  size_t params, grads, am, av, norm, wbf16, Xn, Z[6], Y, dY, dZa, dZb, Xb, Hb1, Hb2, loss, total;
};

MlpLayout mlp_layout(int batch_max) {
  const size_t P = nfm::kMlpNParam, Bp = (size_t)pad16(batch_max), H = nfm::kMlpHid;
  MlpLayout l{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + std::max<size_t>(bytes, 1));
    return o;
  };
  l.params = take(4 * P);
  l.grads = take(4 * P);
  l.am = take(4 * P);
  l.av = take(4 * P);
  l.norm = take(4 * 2 * nfm::kMlpIn);
  l.wbf16 = take(2 * P);
  l.Xn = take(4 * Bp * nfm::kMlpInPad);
  for (int i = 0; i < 6; ++i) l.Z[i] = take(4 * Bp * H);
  l.Y = take(4 * Bp * nfm::kMlpOut);
  l.dY = take(4 * Bp * nfm::kMlpOut);
  l.dZa = take(4 * Bp * H);
  l.dZb = take(4 * Bp * H);
  l.Xb = take(2 * Bp * nfm::kMlpInPad);
  l.Hb1 = take(2 * Bp * H);
  l.Hb2 = take(2 * Bp * H);
  l.loss = take(4 * (1 + 2 * nfm::kMlpLossBlocks));   // the loss, then the partial sums of its reduction
  l.total = off;
  return l;
}

// Scratch of the entry point that allocates nothing (nfm_mlp_infer_bf16_noalloc): the BF16
// activations and the FP32 output rows of one batch of at most kNoAllocRows rows, carved as
// Xb [rows x 96] bf16, H1 and H2 [rows x 128] bf16, Y [rows x 256] float. Every kernel of the
// inference writes all of its buffer's rows (padding included) before any is read, so nothing
// needs clearing between calls. One copy per GPU, held until the process ends; calls that
// overlap on one GPU share it and race.
constexpr int kNoAllocRows = 1024;
constexpr size_t kNoAllocXb = 0;
constexpr size_t kNoAllocH1 = kNoAllocXb + 2 * (size_t)kNoAllocRows * nfm::kMlpInPad;
constexpr size_t kNoAllocH2 = kNoAllocH1 + 2 * (size_t)kNoAllocRows * nfm::kMlpHid;
constexpr size_t kNoAllocY = kNoAllocH2 + 2 * (size_t)kNoAllocRows * nfm::kMlpHid;
constexpr size_t kNoAllocBytes = kNoAllocY + 4 * (size_t)kNoAllocRows * nfm::kMlpOut;
static_assert(kNoAllocH1 % 256 == 0 && kNoAllocH2 % 256 == 0 && kNoAllocY % 256 == 0, "aligned regions");

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_dev[kMaxDevices] = {};

}  // namespace

// In host code this name stands for the array and is not a device address: kernels and copies
// take the address hipGetSymbolAddress returns for the current device (scratch_address()).
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

// The device address of this GPU's copy of the scratch array, looked up once per device with
// that device current (the caller has made it current). nullptr on failure.
char* scratch_address(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    g_scratch_dev[device] = (char*)ptr;
  }
  return g_scratch_dev[device];
}

}  // namespace

struct nfm_mlp {
  int device = 0;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  int batch_max = 0;
  MlpLayout lay{};
  nfm::MlpBuffers buf{};
  int64_t step = 0;  // Adam steps taken
  char* scratch = nullptr;  // this device's no-allocation scratch (device address)
  std::string err;
};

namespace {

nfm_status mfail(nfm_mlp* m, nfm_status s, const std::string& msg) {
  if (m) m->err = msg;
  return s;
}

#define MLP_HIP(m, call)                                                                                \
  do {                                                                                                  \
    hipError_t e_ = (call);                                                                             \
    if (e_ != hipSuccess) return mfail((m), NFM_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define MLP_GUARD(m)                    \
  if (!(m)) return NFM_EINVAL;          \
  if (hipSetDevice((m)->device) != hipSuccess) return mfail((m), NFM_EDEVICE, "hipSetDevice failed")

nfm_status check_batch(nfm_mlp* m, int B, const void* a, const void* b) {
  if (B < 1 || B > m->batch_max) return mfail(m, NFM_EINVAL, "batch must be in [1, batch_max]");
  if (!a || !b) return mfail(m, NFM_EINVAL, "null device pointer");
  return NFM_OK;
}

}  // namespace

extern "C" {

int32_t nfm_mlp_n_params(void) { return nfm::kMlpNParam; }

nfm_status nfm_mlp_workspace_bytes(int32_t batch_max, size_t* bytes) {
  if (!bytes || batch_max < 1 || batch_max > 65536) return NFM_EINVAL;
  *bytes = mlp_layout(batch_max).total;
  return NFM_OK;
}

nfm_status nfm_mlp_create(nfm_mlp** out, int32_t batch_max, void* dev_workspace, size_t workspace_bytes, int device,
                          void* hip_stream) {
  if (!out) return NFM_EINVAL;
  *out = nullptr;
  if (batch_max < 1 || batch_max > 65536 || !dev_workspace || ((uintptr_t)dev_workspace % kAlign) != 0)
    return NFM_EINVAL;
  const MlpLayout l = mlp_layout(batch_max);
  if (workspace_bytes < l.total) return NFM_ESIZE;
  nfm_mlp* m = new (std::nothrow) nfm_mlp();
  if (!m) return NFM_EDEVICE;
  m->device = device;
  m->stream = (hipStream_t)hip_stream;
  m->ws = (char*)dev_workspace;
  m->batch_max = batch_max;
  m->lay = l;
  char* w = m->ws;
  nfm::MlpBuffers& b = m->buf;
  b.params = (float*)(w + l.params);
  b.grads = (float*)(w + l.grads);
  b.adam_m = (float*)(w + l.am);
  b.adam_v = (float*)(w + l.av);
  b.norm = (float*)(w + l.norm);
  b.wbf16 = (uint16_t*)(w + l.wbf16);
  b.Xn = (float*)(w + l.Xn);
  b.Z1 = (float*)(w + l.Z[0]);
  b.A1 = (float*)(w + l.Z[1]);
  b.Z2 = (float*)(w + l.Z[2]);
  b.A2 = (float*)(w + l.Z[3]);
  b.Z3 = (float*)(w + l.Z[4]);
  b.A3 = (float*)(w + l.Z[5]);
  b.Y = (float*)(w + l.Y);
  b.dY = (float*)(w + l.dY);
  b.dZa = (float*)(w + l.dZa);
  b.dZb = (float*)(w + l.dZb);
  b.Xb = (uint16_t*)(w + l.Xb);
  b.Hb1 = (uint16_t*)(w + l.Hb1);
  b.Hb2 = (uint16_t*)(w + l.Hb2);
  b.loss = (float*)(w + l.loss);
  if (hipSetDevice(device) != hipSuccess || hipMemsetAsync(m->ws, 0, l.total, m->stream) != hipSuccess ||
      hipStreamSynchronize(m->stream) != hipSuccess) {
    delete m;
    return NFM_EDEVICE;
  }
  m->scratch = scratch_address(device);   // set-up of the no-allocation entry point, once per device
  if (!m->scratch) {
    delete m;
    return NFM_EDEVICE;
  }
  *out = m;
  return NFM_OK;
}

void nfm_mlp_destroy(nfm_mlp* m) {
  if (!m) return;
  if (hipSetDevice(m->device) == hipSuccess) (void)hipStreamSynchronize(m->stream);
  delete m;
}

const char* nfm_mlp_last_error(const nfm_mlp* m) { return m ? m->err.c_str() : "null context"; }

nfm_status nfm_mlp_init(nfm_mlp* m, uint64_t seed) {
  MLP_GUARD(m);
  MLP_HIP(m, nfm::mlp_init(m->buf, seed, m->stream));
  MLP_HIP(m, hipMemsetAsync(m->buf.grads, 0, 4 * (size_t)nfm::kMlpNParam, m->stream));
  MLP_HIP(m, hipMemsetAsync(m->buf.adam_m, 0, 4 * (size_t)nfm::kMlpNParam, m->stream));
  MLP_HIP(m, hipMemsetAsync(m->buf.adam_v, 0, 4 * (size_t)nfm::kMlpNParam, m->stream));
  float norm[2 * nfm::kMlpIn];
  for (int k = 0; k < nfm::kMlpIn; ++k) {
    norm[k] = 0.f;
    norm[nfm::kMlpIn + k] = 1.f;
  }
  MLP_HIP(m, hipMemcpyAsync(m->buf.norm, norm, sizeof(norm), hipMemcpyHostToDevice, m->stream));
  MLP_HIP(m, hipStreamSynchronize(m->stream));
  m->step = 0;
  return NFM_OK;
}

nfm_status nfm_mlp_set_params(nfm_mlp* m, const float* host_params, const float* host_norm) {
  MLP_GUARD(m);
  if (!host_params && !host_norm) return mfail(m, NFM_EINVAL, "set_params: nothing to set");
  if (host_norm)
    for (int k = 0; k < nfm::kMlpIn; ++k)
      if (!(host_norm[nfm::kMlpIn + k] > 0.f) || !std::isfinite(host_norm[k]))
        return mfail(m, NFM_EINVAL, "set_params: every sd must be positive, every mean finite");
  if (host_params) {
    MLP_HIP(m, hipMemcpyAsync(m->buf.params, host_params, 4 * (size_t)nfm::kMlpNParam, hipMemcpyHostToDevice,
                              m->stream));
    MLP_HIP(m, hipMemsetAsync(m->buf.adam_m, 0, 4 * (size_t)nfm::kMlpNParam, m->stream));
    MLP_HIP(m, hipMemsetAsync(m->buf.adam_v, 0, 4 * (size_t)nfm::kMlpNParam, m->stream));
    m->step = 0;
  }
  if (host_norm)
    MLP_HIP(m, hipMemcpyAsync(m->buf.norm, host_norm, 4 * 2 * (size_t)nfm::kMlpIn, hipMemcpyHostToDevice, m->stream));
  MLP_HIP(m, hipStreamSynchronize(m->stream));
  return NFM_OK;
}

nfm_status nfm_mlp_get_params(nfm_mlp* m, float* host_params, float* host_norm) {
  MLP_GUARD(m);
  if (host_params)
    MLP_HIP(m, hipMemcpyAsync(host_params, m->buf.params, 4 * (size_t)nfm::kMlpNParam, hipMemcpyDeviceToHost,
                              m->stream));
  if (host_norm)
    MLP_HIP(m, hipMemcpyAsync(host_norm, m->buf.norm, 4 * 2 * (size_t)nfm::kMlpIn, hipMemcpyDeviceToHost, m->stream));
  MLP_HIP(m, hipStreamSynchronize(m->stream));
  return NFM_OK;
}

nfm_status nfm_mlp_get_grads(nfm_mlp* m, float* host_grads) {
  MLP_GUARD(m);
  if (!host_grads) return mfail(m, NFM_EINVAL, "get_grads: null pointer");
  MLP_HIP(m, hipMemcpyAsync(host_grads, m->buf.grads, 4 * (size_t)nfm::kMlpNParam, hipMemcpyDeviceToHost, m->stream));
  MLP_HIP(m, hipStreamSynchronize(m->stream));
  return NFM_OK;
}

nfm_status nfm_mlp_forward(nfm_mlp* m, const float* dev_x, int32_t B, float* dev_y) {
  MLP_GUARD(m);
  nfm_status st = check_batch(m, B, dev_x, dev_y);
  if (st != NFM_OK) return st;
  MLP_HIP(m, nfm::mlp_forward_f32(m->buf, dev_x, B, pad16(B), m->buf.Y, m->stream));
  MLP_HIP(m, hipMemcpyAsync(dev_y, m->buf.Y, 4 * (size_t)B * nfm::kMlpOut, hipMemcpyDeviceToDevice, m->stream));
  return NFM_OK;
}

nfm_status nfm_mlp_loss_grad(nfm_mlp* m, const float* dev_x, const float* dev_t, const float* dev_mask, int32_t B,
                             float* host_loss) {
  MLP_GUARD(m);
  nfm_status st = check_batch(m, B, dev_x, dev_t);
  if (st != NFM_OK) return st;
  if (!dev_mask) return mfail(m, NFM_EINVAL, "loss_grad: null mask");
  MLP_HIP(m, nfm::mlp_loss_grad(m->buf, dev_x, dev_t, dev_mask, B, pad16(B), m->stream));
  if (host_loss) {
    MLP_HIP(m, hipMemcpyAsync(host_loss, m->buf.loss, 4, hipMemcpyDeviceToHost, m->stream));
    MLP_HIP(m, hipStreamSynchronize(m->stream));
  }
  return NFM_OK;
}

nfm_status nfm_mlp_adam(nfm_mlp* m, float lr, float beta1, float beta2, float eps) {
  MLP_GUARD(m);
  if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return mfail(m, NFM_EINVAL, "adam: need lr > 0, 0 <= beta < 1, eps > 0");
  const int64_t t = m->step + 1;
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, (double)t)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, (double)t)));
  MLP_HIP(m, nfm::mlp_adam(m->buf, lr, beta1, beta2, eps, c1, c2, m->stream));
  m->step = t;
  return NFM_OK;
}

nfm_status nfm_mlp_train_step(nfm_mlp* m, const float* dev_x, const float* dev_t, const float* dev_mask, int32_t B,
                              float lr) {
  nfm_status st = nfm_mlp_loss_grad(m, dev_x, dev_t, dev_mask, B, nullptr);
  if (st != NFM_OK) return st;
  return nfm_mlp_adam(m, lr, 0.9f, 0.999f, 1e-8f);
}

nfm_status nfm_mlp_last_loss(nfm_mlp* m, float* host_loss) {
  MLP_GUARD(m);
  if (!host_loss) return mfail(m, NFM_EINVAL, "last_loss: null pointer");
  MLP_HIP(m, hipMemcpyAsync(host_loss, m->buf.loss, 4, hipMemcpyDeviceToHost, m->stream));
  MLP_HIP(m, hipStreamSynchronize(m->stream));
  return NFM_OK;
}

nfm_status nfm_mlp_to_bf16(nfm_mlp* m) {
  MLP_GUARD(m);
  MLP_HIP(m, nfm::mlp_to_bf16(m->buf, m->stream));
  return NFM_OK;
}

nfm_status nfm_mlp_infer_bf16(nfm_mlp* m, const float* dev_x, int32_t B, float* dev_y) {
  MLP_GUARD(m);
  nfm_status st = check_batch(m, B, dev_x, dev_y);
  if (st != NFM_OK) return st;
  MLP_HIP(m, nfm::mlp_infer_bf16(m->buf, dev_x, B, pad16(B), m->buf.Y, m->stream));
  MLP_HIP(m, hipMemcpyAsync(dev_y, m->buf.Y, 4 * (size_t)B * nfm::kMlpOut, hipMemcpyDeviceToDevice, m->stream));
  return NFM_OK;
}

nfm_status nfm_mlp_infer_bf16_noalloc(nfm_mlp* m, const float* dev_x, int32_t B, float* dev_y) {
  MLP_GUARD(m);
  if (!dev_x || !dev_y) return mfail(m, NFM_EINVAL, "infer_bf16_noalloc: null device pointer");
  if (B < 1) return mfail(m, NFM_EINVAL, "infer_bf16_noalloc: at least one row");
  if (B > kNoAllocRows)
    return mfail(m, NFM_ERANGE, "infer_bf16_noalloc: at most " + std::to_string(kNoAllocRows) +
                                    " rows per call (the size of the static scratch), got " + std::to_string(B));
  if (!m->scratch) return mfail(m, NFM_ESTATE, "infer_bf16_noalloc: no scratch address for this device");
  nfm::MlpBuffers b = m->buf;   // parameters, normalization and BF16 weights from the network
  b.Xb = (uint16_t*)(m->scratch + kNoAllocXb);
  b.Hb1 = (uint16_t*)(m->scratch + kNoAllocH1);
  b.Hb2 = (uint16_t*)(m->scratch + kNoAllocH2);
  float* Y = (float*)(m->scratch + kNoAllocY);
  MLP_HIP(m, nfm::mlp_infer_bf16(b, dev_x, B, pad16(B), Y, m->stream));
  MLP_HIP(m, hipMemcpyAsync(dev_y, Y, 4 * (size_t)B * nfm::kMlpOut, hipMemcpyDeviceToDevice, m->stream));
  return NFM_OK;
}

}  // extern "C"
