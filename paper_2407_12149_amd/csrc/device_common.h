// Device helpers shared by the MGMC kernels: padded-layout indexing and the
// multilinear transfer weights.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mgmc_internal.h"

namespace mgmc {

constexpr int kBlock = 256;


static __device__ __forceinline__ int64_t pidx(const Geom& g, int i1, int i2, int i3) {
  return int64_t(i1 + 3) + int64_t(g.px) * (int64_t(i2) + int64_t(g.py) * i3);
}

static __device__ __forceinline__ int64_t poff(const Geom& g, int dx, int dy, int dz) {
  return int64_t(dx) + int64_t(g.px) * (int64_t(dy) + int64_t(g.py) * dz);
}

template <int DIM>
static __device__ __forceinline__ void unflatten(int64_t lin, int n, int& i1, int& i2, int& i3) {
  i1 = 1 + int(lin % n);
  lin /= n;
  if (DIM == 3) {
    i2 = 1 + int(lin % n);
    i3 = 1 + int(lin / n);
  } else {
    i2 = 1 + int(lin);
    i3 = 0;
  }
}

static __device__ __forceinline__ double multilinear(int dx, int dy, int dz) {
  double w = 1.0;
  if (dx) w *= 0.5;
  if (dy) w *= 0.5;
  if (dz) w *= 0.5;
  return w;
}


}  // namespace mgmc
