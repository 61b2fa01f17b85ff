// C ABI of the learned prolongation: network evaluation, two-grid loss and
// gradient, and Adam training steps (kernels in kernels_pnet.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>

#include "mgmc.h"
#include "pnet.h"

struct mgmc_pnet {
  mgmc::PnetBuffers B;
  int max_batch = 0;
  int max_errors = 0;
  int step = 0;
  hipStream_t stream = nullptr;
};

namespace {

mgmc_status fail(mgmc_status s, const std::string& m) {
  return static_cast<mgmc_status>(mgmc::record_error(s, m.c_str()));
}

mgmc_status hip_fail(const char* what, hipError_t e) {
  return fail(e == hipErrorOutOfMemory ? MGMC_ENOMEM : MGMC_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

template <class T>
hipError_t dalloc(T*& p, int64_t count) {
  void* raw = nullptr;
  hipError_t e = hipMalloc(&raw, size_t(count) * sizeof(T));
  p = static_cast<T*>(raw);
  return e;
}

void release(mgmc_pnet* p) {
  mgmc::PnetBuffers& B = p->B;
  void* ptrs[] = {B.params, B.grad, B.m, B.v, B.x0, B.z1, B.a1, B.z2, B.a2,
                  B.o, B.d1, B.d2, B.do_, B.w, B.dw, B.loss, B.loss_total};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  delete p;
}

mgmc_status check_batch(const mgmc_pnet* p, int32_t batch) {
  if (!p) return fail(MGMC_EINVAL, "pnet is NULL");
  if (batch < 1 || batch > p->max_batch) return fail(MGMC_EINVAL, "batch must be in [1, max_batch]");
  return MGMC_OK;
}

}  // namespace

extern "C" {

int64_t mgmc_pnet_param_count(void) { return mgmc::pnet_param_count(); }

mgmc_status mgmc_pnet_create(int32_t n, int32_t max_batch, int32_t max_errors, void* hip_stream,
                             mgmc_pnet** out) {
  if (!out) return fail(MGMC_EINVAL, "out is NULL");
  *out = nullptr;
  if (n < 3 || (n & 1) == 0 || n > 8191) return fail(MGMC_EINVAL, "n must be odd, in [3, 8191]");
  if (max_batch < 1 || max_errors < 1) return fail(MGMC_EINVAL, "max_batch and max_errors must be >= 1");
  const int64_t nc = (n - 1) / 2, hw = nc * nc;
  if (int64_t(max_batch) * 24 * hw > (int64_t(1) << 31)) return fail(MGMC_EINVAL, "batch too large");
  mgmc_pnet* p = new (std::nothrow) mgmc_pnet;
  if (!p) return fail(MGMC_ENOMEM, "host allocation failed");
  p->max_batch = max_batch;
  p->max_errors = max_errors;
  p->stream = static_cast<hipStream_t>(hip_stream);
  mgmc::PnetBuffers& B = p->B;
  B.n = n;
  const int64_t np = mgmc::pnet_param_count(), mb = max_batch;
  const int64_t crops = std::max(1, mgmc::pnet_crops_per_field(n));
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = dalloc(B.params, np);
  if (e == hipSuccess) e = dalloc(B.grad, np);
  if (e == hipSuccess) e = dalloc(B.m, np);
  if (e == hipSuccess) e = dalloc(B.v, np);
  if (e == hipSuccess) e = dalloc(B.x0, mb * 24 * hw);
  if (e == hipSuccess) e = dalloc(B.z1, mb * 16 * hw);
  if (e == hipSuccess) e = dalloc(B.a1, mb * 16 * hw);
  if (e == hipSuccess) e = dalloc(B.z2, mb * 16 * hw);
  if (e == hipSuccess) e = dalloc(B.a2, mb * 16 * hw);
  if (e == hipSuccess) e = dalloc(B.o, mb * 9 * hw);
  if (e == hipSuccess) e = dalloc(B.d1, mb * 16 * hw);
  if (e == hipSuccess) e = dalloc(B.d2, mb * 16 * hw);
  if (e == hipSuccess) e = dalloc(B.do_, mb * 9 * hw);
  if (e == hipSuccess) e = dalloc(B.w, mb * 9 * hw);
  if (e == hipSuccess) e = dalloc(B.dw, mb * 9 * hw);
  if (e == hipSuccess) e = dalloc(B.loss, mb * crops);
  if (e == hipSuccess) e = dalloc(B.loss_total, 1);
  if (e == hipSuccess) e = hipMemsetAsync(B.params, 0, size_t(np) * sizeof(float), p->stream);
  if (e == hipSuccess) e = hipMemsetAsync(B.m, 0, size_t(np) * sizeof(float), p->stream);
  if (e == hipSuccess) e = hipMemsetAsync(B.v, 0, size_t(np) * sizeof(float), p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) {
    release(p);
    return hip_fail("pnet allocation", e);
  }
  *out = p;
  return MGMC_OK;
}

mgmc_status mgmc_pnet_set_params(mgmc_pnet* p, const float* params) {
  if (!p || !params) return fail(MGMC_EINVAL, "NULL argument");
  for (int64_t i = 0; i < mgmc::pnet_param_count(); ++i)
    if (!std::isfinite(params[i])) return fail(MGMC_EINVAL, "parameters must be finite");
  const size_t bytes = size_t(mgmc::pnet_param_count()) * sizeof(float);
  hipError_t e = hipMemcpyAsync(p->B.params, params, bytes, hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess) e = hipMemsetAsync(p->B.m, 0, bytes, p->stream);
  if (e == hipSuccess) e = hipMemsetAsync(p->B.v, 0, bytes, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return hip_fail("set_params", e);
  p->step = 0;
  return MGMC_OK;
}

mgmc_status mgmc_pnet_get_params(mgmc_pnet* p, float* params) {
  if (!p || !params) return fail(MGMC_EINVAL, "NULL argument");
  const size_t bytes = size_t(mgmc::pnet_param_count()) * sizeof(float);
  hipError_t e = hipMemcpyAsync(params, p->B.params, bytes, hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return hip_fail("get_params", e);
  return MGMC_OK;
}

mgmc_status mgmc_pnet_weights(mgmc_pnet* p, const double* faces, int32_t batch, double* w) {
  mgmc_status s = check_batch(p, batch);
  if (s != MGMC_OK) return s;
  if (!faces || !w) return fail(MGMC_EINVAL, "NULL argument");
  hipError_t e = mgmc::pnet_forward(p->B, faces, batch, p->stream);
  const int64_t nc = (p->B.n - 1) / 2;
  if (e == hipSuccess)
    e = hipMemcpyAsync(w, p->B.w, size_t(batch) * nc * nc * 9 * sizeof(double), hipMemcpyDeviceToDevice,
                       p->stream);
  if (e != hipSuccess) return hip_fail("pnet forward", e);
  return MGMC_OK;
}

mgmc_status mgmc_pnet_loss_grad(mgmc_pnet* p, const double* faces, const double* errors,
                                int32_t batch, int32_t nerrors, double kappa2, double* loss,
                                float* grad) {
  mgmc_status s = check_batch(p, batch);
  if (s != MGMC_OK) return s;
  if (!faces || !errors) return fail(MGMC_EINVAL, "NULL argument");
  if (nerrors < 1 || nerrors > p->max_errors) return fail(MGMC_EINVAL, "nerrors must be in [1, max_errors]");
  if (mgmc::pnet_crops_per_field(p->B.n) < 1) return fail(MGMC_EINVAL, "grid too small for 15 x 15 coarse crops");
  if (!(kappa2 >= 0.0) || !std::isfinite(kappa2)) return fail(MGMC_EINVAL, "kappa2 must be finite and >= 0");
  hipError_t e = mgmc::pnet_loss_grad(p->B, faces, errors, batch, nerrors, kappa2, p->stream);
  if (e == hipSuccess && loss)
    e = hipMemcpyAsync(loss, p->B.loss_total, sizeof(double), hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess && grad)
    e = hipMemcpyAsync(grad, p->B.grad, size_t(mgmc::pnet_param_count()) * sizeof(float),
                       hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess && (loss || grad)) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return hip_fail("pnet loss/gradient", e);
  return MGMC_OK;
}

mgmc_status mgmc_pnet_train_step(mgmc_pnet* p, const double* faces, const double* errors,
                                 int32_t batch, int32_t nerrors, double kappa2, float lr,
                                 double* loss) {
  if (!(lr > 0.f) || !std::isfinite(lr)) return fail(MGMC_EINVAL, "lr must be positive");
  mgmc_status s = mgmc_pnet_loss_grad(p, faces, errors, batch, nerrors, kappa2, nullptr, nullptr);
  if (s != MGMC_OK) return s;
  p->step += 1;
  hipError_t e = mgmc::pnet_adam(p->B, lr, p->step, p->stream);
  if (e == hipSuccess && loss)
    e = hipMemcpyAsync(loss, p->B.loss_total, sizeof(double), hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess && loss) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return hip_fail("pnet train step", e);
  return MGMC_OK;
}

mgmc_status mgmc_pnet_destroy(mgmc_pnet* p) {
  if (!p) return MGMC_OK;
  hipError_t e = hipStreamSynchronize(p->stream);
  release(p);
  if (e != hipSuccess) return hip_fail("pnet destroy", e);
  return MGMC_OK;
}

}  // extern "C"
