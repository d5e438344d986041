// C ABI of the candidate-proposal network: creation, parameter access,
// inference over feature rows, gradients and Adam training on the device.

#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "chap_internal.h"
#include "mlp_core.h"

using namespace chap;

namespace {

// He-uniform initial parameters: weight p of a layer with fan-in k is
// (2u - 1) sqrt(6 / k) with u = (splitmix64(seed, p) >> 11) 2^-53; biases 0.
std::vector<float> initial_params(uint64_t seed) {
  std::vector<float> w(mlp::kNParam, 0.0f);
  auto fill = [&](int off, int count, int fan_in) {
    const double lim = std::sqrt(6.0 / (double)fan_in);
    for (int p = off; p < off + count; ++p) {
      const double u = (double)(splitmix64(seed, (uint64_t)p) >> 11) * 0x1.0p-53;
      w[p] = (float)((2.0 * u - 1.0) * lim);
    }
  };
  fill(mlp::kOffW1, mlp::kHid * mlp::kIn, mlp::kIn);
  fill(mlp::kOffW2, mlp::kHid * mlp::kHid, mlp::kHid);
  fill(mlp::kOffW3, mlp::kHid, mlp::kHid);
  return w;
}

int upload_params(chap_model* M, const float* host) {
  for (int p = 0; p < mlp::kNParam; ++p)
    if (!std::isfinite(host[p])) return fail(CHAP_EINVAL, "non-finite parameter at " + std::to_string(p));
  CHAP_HIP(hipMemcpy(M->dev.w, host, sizeof(float) * mlp::kNParam, hipMemcpyHostToDevice));
  CHAP_HIP(hipMemset(M->dev.m, 0, sizeof(float) * mlp::kNParam));
  CHAP_HIP(hipMemset(M->dev.v, 0, sizeof(float) * mlp::kNParam));
  const double adam0[3] = {1.0, 1.0, 0.0};
  CHAP_HIP(hipMemcpy(M->dev.adam, adam0, sizeof(adam0), hipMemcpyHostToDevice));
  CHAP_HIP(launch_mlp_bf16_copy(M->dev, nullptr));
  CHAP_HIP(hipDeviceSynchronize());
  return CHAP_OK;
}

int check_device(const chap_model* M, const char* who) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(CHAP_EHIP, std::string(who) + ": hipGetDevice failed");
  if (dev != M->device) return fail(CHAP_EINVAL, std::string(who) + ": model lives on another device");
  return CHAP_OK;
}

}  // namespace

extern "C" {

int chap_model_create(chap_model** out, uint64_t seed) {
  if (!out) return fail(CHAP_EINVAL, "chap_model_create: null output");
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count == 0) return fail(CHAP_ENOTBUILT, "no HIP device visible");
  std::unique_ptr<chap_model> M(new chap_model());
  CHAP_HIP(hipGetDevice(&M->device));
  DeviceArena& A = M->arena;
  ModelDev& D = M->dev;
  CHAP_HIP(A.alloc(&D.w, mlp::kNParam));
  CHAP_HIP(A.alloc(&D.wb, mlp::kNParam));
  CHAP_HIP(A.alloc(&D.m, mlp::kNParam));
  CHAP_HIP(A.alloc(&D.v, mlp::kNParam));
  CHAP_HIP(A.alloc(&D.adam, 3));
  CHAP_HIP(A.alloc(&D.grad, mlp::kNParam));
  CHAP_HIP(A.alloc(&D.partials, (size_t)kGradBlocks * kNParamPad));
  const std::vector<float> w = initial_params(seed);
  const int rc = upload_params(M.get(), w.data());
  if (rc != CHAP_OK) return rc;
  *out = M.release();
  return CHAP_OK;
}

void chap_model_destroy(chap_model* m) { delete m; }

int chap_model_get_params(const chap_model* m, float* params) {
  if (!m || !params) return fail(CHAP_EINVAL, "chap_model_get_params: null argument");
  CHAP_HIP(hipDeviceSynchronize());
  CHAP_HIP(hipMemcpy(params, m->dev.w, sizeof(float) * mlp::kNParam, hipMemcpyDeviceToHost));
  return CHAP_OK;
}

int chap_model_set_params(chap_model* m, const float* params) {
  if (!m || !params) return fail(CHAP_EINVAL, "chap_model_set_params: null argument");
  const int rc = check_device(m, "chap_model_set_params");
  if (rc != CHAP_OK) return rc;
  return upload_params(m, params);
}

int chap_model_forward(chap_model* m, const uint16_t* d_feat, int64_t n, float* d_out, void* hip_stream) {
  if (!m || n < 0 || (n > 0 && (!d_feat || !d_out))) return fail(CHAP_EINVAL, "chap_model_forward: bad argument");
  const int rc = check_device(m, "chap_model_forward");
  if (rc != CHAP_OK) return rc;
  CHAP_HIP(launch_mlp_forward(m->dev, d_feat, n, d_out, (hipStream_t)hip_stream));
  return CHAP_OK;
}

int chap_model_grad(chap_model* m, const uint16_t* d_feat, const float* d_target, int64_t n, float* d_grad,
                    void* hip_stream) {
  if (!m || n <= 0 || !d_feat || !d_target || !d_grad) return fail(CHAP_EINVAL, "chap_model_grad: bad argument");
  if (n > (int64_t)1 << 40) return fail(CHAP_EINVAL, "chap_model_grad: too many samples");
  const int rc = check_device(m, "chap_model_grad");
  if (rc != CHAP_OK) return rc;
  hipStream_t s = (hipStream_t)hip_stream;
  CHAP_HIP(launch_mlp_grad(m->dev, d_feat, d_target, n, n, 0, 0, 0, s));
  CHAP_HIP(launch_mlp_reduce(m->dev, n, 0, 0.0f, s));
  CHAP_HIP(hipMemcpyAsync(d_grad, m->dev.grad, sizeof(float) * mlp::kNParam, hipMemcpyDeviceToDevice, s));
  return CHAP_OK;
}

int chap_model_train(chap_model* m, const uint16_t* d_feat, const float* d_target, int64_t npairs, int32_t steps,
                     int32_t batch, float lr, uint64_t seed, void* hip_stream) {
  if (!m || npairs <= 0 || !d_feat || !d_target || steps < 0 || batch <= 0 || !(lr > 0.0f) || !std::isfinite(lr))
    return fail(CHAP_EINVAL, "chap_model_train: bad argument");
  const int rc = check_device(m, "chap_model_train");
  if (rc != CHAP_OK) return rc;
  hipStream_t s = (hipStream_t)hip_stream;
  for (int32_t k = 0; k < steps; ++k) {
    CHAP_HIP(launch_mlp_grad(m->dev, d_feat, d_target, npairs, batch, 1, seed, (uint64_t)k * (uint64_t)batch, s));
    CHAP_HIP(launch_mlp_reduce(m->dev, batch, 1, lr, s));
  }
  return CHAP_OK;
}

}  // extern "C"
