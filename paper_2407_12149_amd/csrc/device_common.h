// Device helpers shared by the MGMC kernels: padded-layout indexing and the
// multilinear transfer weights.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mgmc_internal.h"

namespace mgmc {

constexpr int kBlock = 256;


static __device__ __forceinline__ int64_t pidx(const Geom& g, int i1, int i2, int i3) {
  return g.o0 + int64_t(i1 + 3) + int64_t(g.px) * (int64_t(i2) + int64_t(g.py) * i3);
}

// (B_{l-1} v)(J) for chain c at the coarse site whose row of B_{l-1} is r
// (r < 0: no observation touches the site).
static __device__ __forceinline__ double lowrank_rhs_row(const LowRankRhs& lr, int c, int r) {
  if (r < 0) return 0.0;
  double s = 0.0;
  for (int64_t e = lr.ptr[r]; e < lr.ptr[r + 1]; ++e)
    s += lr.val[e] * lr.v[int64_t(c) * lr.beta + lr.col[e]];
  return s;
}

// Row of B_{l-1} at coarse padded site iJ, or -1 (also without a low-rank term).
static __device__ __forceinline__ int lowrank_row(const LowRankRhs& lr, int64_t iJ) {
  return lr.row_of == nullptr ? -1 : lr.row_of[iJ];
}

// (B_{l-1} v)(J) for coarse padded site iJ and chain c (0 without a low-rank term).
static __device__ __forceinline__ double lowrank_rhs(const LowRankRhs& lr, int c, int64_t iJ) {
  return lowrank_rhs_row(lr, c, lowrank_row(lr, iJ));
}

static __device__ __forceinline__ int64_t poff(const Geom& g, int dx, int dy, int dz) {
  return int64_t(dx) + int64_t(g.px) * (int64_t(dy) + int64_t(g.py) * dz);
}

// Stencil entry t of the interior padded site i.  Past the centre the entry
// is read as the opposite entry of the neighbour i + delta(t) (the operators
// are symmetric entry by entry), so only the centre and the entries towards
// lower indices come from memory.  The neighbour may be a ghost position,
// whose entries are zero, as is the state they would multiply.
template <typename T, int DIM>
static __device__ __forceinline__ T stencil_entry(const T* __restrict__ coef, const Geom& g, int t,
                                                  int64_t i) {
  constexpr int S = DIM == 2 ? 9 : 27;
  if (t <= S / 2) return coef[int64_t(t) * g.Np + i];
  const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = DIM == 3 ? t / 9 - 1 : 0;
  return coef[int64_t(S - 1 - t) * g.Np + i + poff(g, dx, dy, dz)];
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
