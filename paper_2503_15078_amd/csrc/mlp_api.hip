// C-ABI of the warm-start network's trainer: float32 master weights and Adam moments on
// the device, training batches and inputs in device memory (any allocator, e.g. torch).
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "device.hpp"
#include "status.hpp"

struct lg_mlp {
  float *P = nullptr, *M = nullptr, *V = nullptr;  // parameters, Adam moments
  float* partial = nullptr;                          // [kMlpMaxBlocks][kMlpParams + 1]
  float* out = nullptr;                              // [kMlpParams + 1]: gradient, loss
  long step = 0;
};

namespace {

#define MCHK(x)                                                                      \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess) {                                                          \
      lg::set_error(std::string("HIP error: ") + hipGetErrorString(e_) + " at " #x); \
      return SIM_E_DEVICE;                                                           \
    }                                                                                \
  } while (0)

void release(lg_mlp* m) {
  for (float* p : {m->P, m->M, m->V, m->partial, m->out})
    if (p) (void)hipFree(p);
  delete m;
}

// the kernels read features (and parameters) as float4
bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

int check_batch(lg_mlp* m, const float* x, const float* t, int32_t n, bool need_t) {
  if (!m || !x || (need_t && !t) || n <= 0 || (need_t && n > lg::kMlpMaxBatch) || !aligned16(x)) {
    lg::set_error("bad arguments");
    return SIM_E_ARG;
  }
  return SIM_OK;
}

// training launch + reduction (+ Adam when lr > 0 and update)
int run_step(lg_mlp* m, const float* x, const float* t, int32_t n, float lr, int update, hipStream_t st) {
  lg::launch_mlp_train(m->P, x, t, n, m->partial, st);
  const float b1 = 0.9f, b2 = 0.999f;
  float c1 = 1.0f, c2 = 1.0f;
  if (update) {
    ++m->step;
    c1 = (float)(1.0 / (1.0 - std::pow((double)b1, (double)m->step)));
    c2 = (float)(1.0 / (1.0 - std::pow((double)b2, (double)m->step)));
  }
  lg::launch_mlp_adam(m->P, m->M, m->V, m->partial, n, lr, b1, b2, 1e-8f, c1, c2, update, update ? nullptr : m->out,
                      m->out + lg::kMlpParams, st);
  MCHK(hipGetLastError());
  return SIM_OK;
}

// ---- fixed scratch of the no-allocation gradient
// The per-block partial sums of one gradient launch live in a file-scope device array,
// one copy per GPU, held until the process ends.  Host code must not pass the array's
// name to a kernel (on the host it only names a stand-in); it passes the device address
// that hipGetSymbolAddress returned for the current device.
constexpr int kNoAllocMaxBlocks = 64;  // 64 samples per block: batches of at most 4096
constexpr int kNoAllocMaxDevices = 64;
static_assert(kNoAllocMaxBlocks * 64 == SIM_MLP_NOALLOC_MAX_BATCH, "batch limit of the header");

__device__ __align__(256) float scratch[(size_t)kNoAllocMaxBlocks * (lg::kMlpParams + 1)];

std::mutex g_scratch_mu;
float* g_scratch_ptr[kNoAllocMaxDevices] = {};

// Device address of the current device's scratch array (looked up once per device).
int scratch_of_current_device(float** out) {
  int dev = -1;
  MCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoAllocMaxDevices) {
    lg::set_error("mlp_gradient_noalloc: device index out of range");
    return SIM_E_DEVICE;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      lg::set_error(std::string("mlp_gradient_noalloc: hipGetSymbolAddress failed: ") + hipGetErrorString(e));
      return SIM_E_DEVICE;
    }
    g_scratch_ptr[dev] = static_cast<float*>(p);
  }
  *out = g_scratch_ptr[dev];
  return SIM_OK;
}

}  // namespace

extern "C" {

int mlp_create(const float* params, int32_t n_params, mlp_t* out) {
  if (!params || !out || n_params != lg::kMlpParams) {
    lg::set_error("mlp_create: expected " + std::to_string(lg::kMlpParams) + " parameters");
    return SIM_E_ARG;
  }
  *out = nullptr;
  lg_mlp* m = new (std::nothrow) lg_mlp();
  if (!m) return SIM_E_NOMEM;
  const size_t np = lg::kMlpParams;
  if (hipMalloc(&m->P, np * 4) != hipSuccess || hipMalloc(&m->M, np * 4) != hipSuccess ||
      hipMalloc(&m->V, np * 4) != hipSuccess || hipMalloc(&m->out, (np + 1) * 4) != hipSuccess ||
      hipMalloc(&m->partial, (size_t)lg::kMlpMaxBlocks * (np + 1) * 4) != hipSuccess) {
    release(m);
    lg::set_error("mlp_create: device allocation failed");
    return SIM_E_NOMEM;
  }
  // the null-stream fills are waited for: training runs on the caller's stream, which may
  // be non-blocking and so unordered with them
  if (hipMemcpy(m->P, params, np * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(m->M, 0, np * 4) != hipSuccess || hipMemset(m->V, 0, np * 4) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    release(m);
    lg::set_error("mlp_create: upload failed");
    return SIM_E_DEVICE;
  }
  *out = m;
  return SIM_OK;
}

int mlp_set_params(mlp_t m, const float* params, int32_t n_params) {
  if (!m || !params || n_params != lg::kMlpParams) {
    lg::set_error("bad arguments");
    return SIM_E_ARG;
  }
  MCHK(hipDeviceSynchronize());  // no training step of the caller's stream still reads them
  MCHK(hipMemcpy(m->P, params, (size_t)n_params * 4, hipMemcpyHostToDevice));
  MCHK(hipMemset(m->M, 0, (size_t)n_params * 4));
  MCHK(hipMemset(m->V, 0, (size_t)n_params * 4));
  MCHK(hipDeviceSynchronize());
  m->step = 0;
  return SIM_OK;
}

int mlp_get_params(mlp_t m, float* params, int32_t n_params) {
  if (!m || !params || n_params != lg::kMlpParams) {
    lg::set_error("bad arguments");
    return SIM_E_ARG;
  }
  MCHK(hipDeviceSynchronize());
  MCHK(hipMemcpy(params, m->P, (size_t)n_params * 4, hipMemcpyDeviceToHost));
  return SIM_OK;
}

int mlp_forward(mlp_t m, const float* d_x, float* d_y, int32_t n, void* hip_stream) {
  if (check_batch(m, d_x, d_y, n, false) != SIM_OK || !d_y) return SIM_E_ARG;
  lg::launch_mlp_forward(m->P, d_x, d_y, n, reinterpret_cast<hipStream_t>(hip_stream));
  MCHK(hipGetLastError());
  return SIM_OK;
}

int mlp_train_step(mlp_t m, const float* d_x, const float* d_t, int32_t n, float lr, void* hip_stream, float* loss) {
  if (check_batch(m, d_x, d_t, n, true) != SIM_OK || !(lr > 0.0f)) {
    lg::set_error("bad arguments");
    return SIM_E_ARG;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  int rc = run_step(m, d_x, d_t, n, lr, 1, st);
  if (rc != SIM_OK) return rc;
  if (loss) {
    MCHK(hipMemcpyAsync(loss, m->out + lg::kMlpParams, 4, hipMemcpyDeviceToHost, st));
    MCHK(hipStreamSynchronize(st));
  }
  return SIM_OK;
}

int mlp_gradient(mlp_t m, const float* d_x, const float* d_t, int32_t n, void* hip_stream, float* grad, float* loss) {
  if (check_batch(m, d_x, d_t, n, true) != SIM_OK || !grad || !loss) {
    lg::set_error("bad arguments");
    return SIM_E_ARG;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  int rc = run_step(m, d_x, d_t, n, 0.0f, 0, st);
  if (rc != SIM_OK) return rc;
  MCHK(hipMemcpyAsync(grad, m->out, (size_t)lg::kMlpParams * 4, hipMemcpyDeviceToHost, st));
  MCHK(hipMemcpyAsync(loss, m->out + lg::kMlpParams, 4, hipMemcpyDeviceToHost, st));
  MCHK(hipStreamSynchronize(st));
  return SIM_OK;
}

int mlp_gradient_noalloc(const float* d_params, const float* d_x, const float* d_t, int32_t n, float* d_out,
                         void* hip_stream) {
  if (!d_params || !d_x || !d_t || !d_out || n <= 0 || n > SIM_MLP_NOALLOC_MAX_BATCH || !aligned16(d_params) ||
      !aligned16(d_x)) {
    lg::set_error("mlp_gradient_noalloc: bad arguments (batch must hold 1.." +
                  std::to_string(SIM_MLP_NOALLOC_MAX_BATCH) + " samples; params and features 16-byte aligned)");
    return SIM_E_ARG;
  }
  float* part = nullptr;
  int rc = scratch_of_current_device(&part);
  if (rc != SIM_OK) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  // the training kernel writes every entry of its blocks' partial rows, so the scratch
  // left by an earlier call needs no clearing; the reduction only reads parameters when
  // it updates them, which it does not here
  lg::launch_mlp_train(d_params, d_x, d_t, n, part, st);
  lg::launch_mlp_adam(nullptr, nullptr, nullptr, part, n, 0.0f, 0.9f, 0.999f, 1e-8f, 1.0f, 1.0f, 0, d_out,
                      d_out + lg::kMlpParams, st);
  MCHK(hipGetLastError());
  return SIM_OK;
}

int mlp_destroy(mlp_t m) {
  if (!m) return SIM_E_ARG;
  (void)hipDeviceSynchronize();
  release(m);
  return SIM_OK;
}

}  // extern "C"
