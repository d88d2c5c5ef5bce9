// C-ABI of the warm-start network's trainer: float32 master weights and Adam moments on
// the device, training batches and inputs in device memory (any allocator, e.g. torch).
#include <hip/hip_runtime.h>

#include <cmath>
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

int check_batch(lg_mlp* m, const float* x, const float* t, int32_t n, bool need_t) {
  if (!m || !x || (need_t && !t) || n <= 0 || (need_t && n > lg::kMlpMaxBatch)) {
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

int mlp_destroy(mlp_t m) {
  if (!m) return SIM_E_ARG;
  (void)hipDeviceSynchronize();
  release(m);
  return SIM_OK;
}

}  // extern "C"
