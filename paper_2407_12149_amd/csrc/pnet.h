// Device buffers and host launchers of the learned-prolongation network.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mgmc {

// All pointers are device memory owned by the caller of the launchers.
struct PnetBuffers {
  int n = 0;               // fine interior nodes per axis (odd); coarse nc = (n-1)/2
  float* params = nullptr; // network parameters, pnet_param_count() floats
  float* grad = nullptr;   // gradient of the loss, same layout
  float* m = nullptr;      // Adam first moment
  float* v = nullptr;      // Adam second moment
  float* x0 = nullptr;     // features [batch][24][nc][nc]
  float* z1 = nullptr;     // pre-activations and activations [batch][16][nc][nc]
  float* a1 = nullptr;
  float* z2 = nullptr;
  float* a2 = nullptr;
  float* o = nullptr;      // outputs [batch][9][nc][nc]
  float* d1 = nullptr;     // back-propagated signals [batch][16][nc][nc]
  float* d2 = nullptr;
  float* do_ = nullptr;    // [batch][9][nc][nc]
  double* w = nullptr;     // prolongation weights [batch][nc*nc][9]
  double* dw = nullptr;    // d loss / d w, same layout
  double* loss = nullptr;  // per crop losses [batch][crops], then the total at loss_total
  double* loss_total = nullptr;
};

int64_t pnet_param_count();
int pnet_crops_per_field(int n);
hipError_t pnet_forward(const PnetBuffers& P, const double* faces, int batch, hipStream_t st);
hipError_t pnet_loss_grad(const PnetBuffers& P, const double* faces, const double* errors,
                          int batch, int K, double kappa2, hipStream_t st);
hipError_t pnet_adam(const PnetBuffers& P, float lr, int step, hipStream_t st);

}  // namespace mgmc

namespace mgmc {
// Records msg as this thread's last error and returns status.
int record_error(int status, const char* msg);
}  // namespace mgmc
