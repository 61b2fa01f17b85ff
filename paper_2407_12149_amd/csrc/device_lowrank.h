// The vectors of the low-rank step of the random smoother (Alg. 3) after a
// 2D sweep that wrote its snapshot of B's sites: for chain c and observation j
//   xi_j = Gamma_jj^{-1/2} zeta_j,   t_j = (B^T theta*)_j - Gamma_jj xi_j,
// with theta* the swept state and zeta_j standard normal (Philox counter
// (pair j / 2, word, m, 1), Box-Muller pair element j % 2).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_rng.h"

namespace mgmc {

// Forms (t, xi) for chains c0 .. c0 + nc - 1 and hands every observation j
// and chain slot cc < ncs to put(j, cc, t, xi), with zeros for the slots
// cc >= nc.  All threads of the block take part.  The snapshot holds B's
// weight times the swept value in KP slots per observation
// ([chain][beta][KP], zero padded); each sum takes its slots in order, CH
// slots of each of a thread's two observations loaded together.
template <int KP, int CH = KP, class Put>
__device__ __forceinline__ void lowrank_t_xi(const double* __restrict__ bsnap, int64_t bslots,
                                             int beta, const double* __restrict__ gisq,
                                             const double* __restrict__ gam, uint32_t word,
                                             uint32_t m, uint32_t seed, uint32_t chain0, int c0,
                                             int nc, int ncs, Put put) {
  const int npairs = (beta + 1) / 2;
  for (int task = threadIdx.x; task < npairs * ncs; task += blockDim.x) {
    const int p = task % npairs, cc = task / npairs;
    double tv[2] = {0.0, 0.0}, xv[2] = {0.0, 0.0};
    if (cc < nc) {
      const int c = c0 + cc;
      const double* sn = bsnap + int64_t(c) * bslots;
      double w[2] = {0.0, 0.0};
      int64_t e0[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) e0[h] = int64_t(min(2 * p + h, beta - 1)) * KP;
#pragma unroll 1
      for (int u0 = 0; u0 < KP; u0 += CH) {
        double pr[2][CH];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int u = 0; u < CH; ++u) pr[h][u] = sn[e0[h] + u0 + u];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int u = 0; u < CH; ++u) w[h] += pr[h][u];
      }
      const Block4 blk = philox10(uint32_t(p), word, m, 1u, seed, chain0 + c);
      double z[2];
      Gauss<double>::pair(blk, z[0], z[1]);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int j = min(2 * p + h, beta - 1);
        xv[h] = z[h] * gisq[j];
        tv[h] = w[h] - gam[j] * xv[h];
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int j = 2 * p + h;
      if (j < beta) put(j, cc, tv[h], xv[h]);
    }
  }
}

}  // namespace mgmc
