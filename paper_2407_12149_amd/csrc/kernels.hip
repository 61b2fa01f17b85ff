// HIP kernels of one MGMC update (gfx950).
//
//  * k_sweep: one colour pass of the random Gauss-Seidel smoother (Alg. 2/3
//    with M = D + L in colour order, omega = 1): for every site i of the colour
//    theta_i <- (f_i - sum_{j != i} A_ij theta_j) / A_ii + z_i / sqrt(A_ii),
//    z_i from Philox.  One thread owns one Philox block, i.e. the two sites of
//    the colour at x-distance 2 that share it.
//  * k_restrict: f_{l-1}(J) = sum_delta w_J(delta) (f - A theta)(2J + delta),
//    the restricted residual with R = P^T (Alg. 1, restriction step).
//  * k_prolong: theta_i += sum_J P_iJ psi_J (Alg. 1, prolongation step).
//  * k_coarsest: theta_0 = K f_0 + U^{-1} z, an exact draw from
//    N(At_0^{-1} f_0, At_0^{-1}) (Sec. 3.5).
//  * k_lowrank_*: the low-rank correction of Alg. 3 (see k_lowrank_prep).
//  * k_qoi_*: q = F^T theta per chain, fixed-order reductions.
#include <algorithm>

#include "device_common.h"
#include "device_lowrank.h"
#include "device_rng.h"
#include "mgmc_internal.h"

namespace mgmc {

Geom make_geom(int dim, int n, int halo) {
  Geom g;
  g.n = n;
  if (halo == 2) {
    g.px = ((n + 6) + 3) / 4 * 4;
    g.py = n + 4;
    g.o0 = g.px;
    g.Np = int64_t(g.px) * g.py;
    return g;
  }
  g.px = ((n + 5) + 3) / 4 * 4;
  g.py = n + 2;
  g.Np = int64_t(g.px) * g.py * (dim == 3 ? (n + 2) : 1);
  return g;
}

namespace {

// Relaxed site update of the random SOR sweep (Sec. 3.3, eq. SOR_smoother;
// noise covariance (2 - omega)/omega D, eq. low_rank_smoother_covariance):
// (1 - omega) theta_i + omega s / A_ii + sqrt(omega (2 - omega) / A_ii) z.
template <typename T>
__device__ __forceinline__ T sor_site(T old, T s, T ivd, T isd, T z, T om) {
  return (T(1) - om) * old + om * (s * ivd) + sqrt(om * (T(2) - om)) * isd * z;
}

// One Gauss-Seidel site update (neighbours in ascending index order).
template <typename T, int DIM, bool CROSS>
__device__ __forceinline__ void gs_update(const T* __restrict__ coef, const T* __restrict__ invd,
                                          const T* __restrict__ isqd, T* __restrict__ th,
                                          const T* __restrict__ f, const Geom& g, int64_t i, T z) {
  constexpr int S = DIM == 2 ? 9 : 27;
  T s = f ? f[i] : T(0);
#pragma unroll
  for (int t = 0; t < S; ++t) {
    const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = DIM == 3 ? t / 9 - 1 : 0;
    const int nz = (dx != 0) + (dy != 0) + (dz != 0);
    if (nz == 0 || (CROSS && nz != 1)) continue;
    s -= stencil_entry<T, DIM>(coef, g, t, i) * th[i + poff(g, dx, dy, dz)];
  }
  th[i] = s * invd[i] + z * isqd[i];
}

template <typename T, int DIM, bool CROSS>
__global__ __launch_bounds__(kBlock) void k_sweep(const T* __restrict__ coef,
                                                  const T* __restrict__ invd,
                                                  const T* __restrict__ isqd, T* __restrict__ theta,
                                                  const T* __restrict__ f, int64_t fcs, Geom g,
                                                  int colour, uint32_t word,
                                                  const int64_t* __restrict__ mcur, uint32_t seed,
                                                  uint32_t chain0, int cpb, int nchains, T om) {
  constexpr int S = DIM == 2 ? 9 : 27;
  constexpr int NB = CROSS ? 2 * DIM : S - 1;  // neighbours per site
  const int p1 = colour & 1, p2 = (colour >> 1) & 1, p3 = (colour >> 2) & 1;
  const int n = g.n;
  const int m1 = p1 ? (n + 1) / 2 : (n - 1) / 2;
  const int m2 = p2 ? (n + 1) / 2 : (n - 1) / 2;
  const int m3 = DIM == 3 ? (p3 ? (n + 1) / 2 : (n - 1) / 2) : 1;
  const int qx = (m1 + 1) / 2;
  const int64_t total = int64_t(qx) * m2 * m3;
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= total) return;
  const int q = int(gid % qx);
  const int64_t rest = gid / qx;
  const int s2 = int(rest % m2), s3 = int(rest / m2);
  const int i1 = 4 * q + (p1 ? 1 : 2);
  const int i2 = 2 * s2 + (p2 ? 1 : 2);
  const int i3 = DIM == 3 ? 2 * s3 + (p3 ? 1 : 2) : 0;
  const uint32_t pair = uint32_t(q) + uint32_t(qx) * (uint32_t(s2) + uint32_t(m2) * uint32_t(s3));
  const uint32_t m = uint32_t(*mcur);
  const bool two = 2 * q + 1 < m1;
  const int64_t ia = pidx(g, i1, i2, i3);
  // the stencil of the pair's two sites, in registers for the chain group
  // (neighbours in ascending index order)
  T cf[2][NB], ivd[2], isd[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const bool in = k == 0 || two;
    int b = 0;
#pragma unroll
    for (int t = 0; t < S; ++t) {
      const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = DIM == 3 ? t / 9 - 1 : 0;
      const int nz = (dx != 0) + (dy != 0) + (dz != 0);
      if (nz == 0 || (CROSS && nz != 1)) continue;
      cf[k][b++] = in ? stencil_entry<T, DIM>(coef, g, t, ia + 2 * k) : T(0);
    }
    ivd[k] = in ? invd[ia + 2 * k] : T(0);
    isd[k] = sqrt(ivd[k]);  // A_ii^{-1/2} from the inverse diagonal (0 where absent)
  }
  const int cb = int(blockIdx.y) * cpb;
  const int ce = min(nchains, cb + cpb);
  for (int c = cb; c < ce; ++c) {
    T* th = theta + int64_t(c) * g.Np;
    // Both sites' neighbour loads are issued before the noise is drawn and
    // without branches: a missing second site (past the row end) reads
    // padding and ghost entries, which stay in bounds, and is not stored.
    T s[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int64_t i = ia + 2 * k;
      s[k] = f ? f[int64_t(c) * fcs + i] : T(0);
      int b = 0;
#pragma unroll
      for (int t = 0; t < S; ++t) {
        const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = DIM == 3 ? t / 9 - 1 : 0;
        const int nz = (dx != 0) + (dy != 0) + (dz != 0);
        if (nz == 0 || (CROSS && nz != 1)) continue;
        s[k] -= cf[k][b++] * th[i + poff(g, dx, dy, dz)];
      }
    }
    const Block4 blk = philox10(pair, word | uint32_t(colour), m, 0u, seed, chain0 + c);
    T z[2];
    Gauss<T>::pair(blk, z[0], z[1]);
    if (om == T(1)) {
      th[ia] = s[0] * ivd[0] + z[0] * isd[0];
      if (two) th[ia + 2] = s[1] * ivd[1] + z[1] * isd[1];
    } else {
      th[ia] = sor_site(th[ia], s[0], ivd[0], isd[0], z[0], om);
      if (two) th[ia + 2] = sor_site(th[ia + 2], s[1], ivd[1], isd[1], z[1], om);
    }
  }
}

// Parity pass of a 3D 7-point sweep: all colours with parity sum `parity`
// (they never couple through axis neighbours), one thread per Philox pair of
// the row's colour.  Equivalent to the four colour passes of that parity.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_sweep_parity3d(const T* __restrict__ coef,
                                                           const T* __restrict__ invd,
                                                           const T* __restrict__ isqd,
                                                           T* __restrict__ theta,
                                                           const T* __restrict__ f, int64_t fcs,
                                                           Geom g, int parity, uint32_t word,
                                                           const int64_t* __restrict__ mcur,
                                                           uint32_t seed, uint32_t chain0, int cpb,
                                                           int nchains, T om) {
  const int n = g.n;
  const int qmax = ((n + 1) / 2 + 1) / 2;  // pairs per row for the odd x-sublattice
  const int64_t total = int64_t(qmax) * n * n;
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= total) return;
  const int q = int(gid % qmax);
  const int64_t row = gid / qmax;
  const int i2 = 1 + int(row % n), i3 = 1 + int(row / n);
  const int xpar = (parity + i2 + i3) & 1;  // x parity giving parity sum `parity`
  const int colour = xpar | ((i2 & 1) << 1) | ((i3 & 1) << 2);
  const int m1 = xpar ? (n + 1) / 2 : (n - 1) / 2;
  const int qx = (m1 + 1) / 2;
  if (q >= qx) return;
  const int m2 = (i2 & 1) ? (n + 1) / 2 : (n - 1) / 2;
  const int s2 = (i2 - 1) >> 1, s3 = (i3 - 1) >> 1;
  const uint32_t pair = uint32_t(q) + uint32_t(qx) * (uint32_t(s2) + uint32_t(m2) * uint32_t(s3));
  const uint32_t m = uint32_t(*mcur);
  const int i1 = 4 * q + (xpar ? 1 : 2);
  const bool two = 2 * q + 1 < m1;
  // the stencil of the pair's two sites, kept in registers for every chain
  // of the block's group: axis neighbours in ascending index order
  const int64_t ia = pidx(g, i1, i2, i3);
  const int64_t off[6] = {-int64_t(g.px) * g.py, -int64_t(g.px), -1, 1, int64_t(g.px),
                          int64_t(g.px) * g.py};
  const int tix[6] = {4, 10, 12, 14, 16, 22};
  T cf[2][6], ivd[2], isd[2], rhs[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int64_t i = ia + 2 * k;
    const bool in = k == 0 || two;
#pragma unroll
    // +x, +y, +z entries from the neighbour's opposite entry (symmetric operator)
    for (int e = 0; e < 6; ++e)
      cf[k][e] = in ? coef[int64_t(tix[e < 3 ? e : 5 - e]) * g.Np + i + (e < 3 ? 0 : off[e])] : T(0);
    ivd[k] = in ? invd[i] : T(0);
    isd[k] = sqrt(ivd[k]);  // A_ii^{-1/2} from the inverse diagonal (0 where absent)
    rhs[k] = (in && f && fcs == 0) ? f[i] : T(0);
  }
  const int cb = int(blockIdx.y) * cpb;
  const int ce = min(nchains, cb + cpb);
  for (int c = cb; c < ce; ++c) {
    T* th = theta + int64_t(c) * g.Np;
    // neighbour loads first and branch-free (a missing second site reads
    // padding and ghost entries and is not stored), then the noise
    T s[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int64_t i = ia + 2 * k;
      s[k] = (f && fcs != 0) ? f[int64_t(c) * fcs + i] : rhs[k];
#pragma unroll
      for (int e = 0; e < 6; ++e) s[k] -= cf[k][e] * th[i + off[e]];
    }
    const Block4 blk = philox10(pair, word | uint32_t(colour), m, 0u, seed, chain0 + c);
    T z[2];
    Gauss<T>::pair(blk, z[0], z[1]);
    if (om == T(1)) {
      th[ia] = s[0] * ivd[0] + z[0] * isd[0];
      if (two) th[ia + 2] = s[1] * ivd[1] + z[1] * isd[1];
    } else {
      th[ia] = sor_site(th[ia], s[0], ivd[0], isd[0], z[0], om);
      if (two) th[ia + 2] = sor_site(th[ia + 2], s[1], ivd[1], isd[1], z[1], om);
    }
  }
}

template <typename T, int DIM, bool CROSS, bool USERP>
__global__ __launch_bounds__(kBlock) void k_restrict(const T* __restrict__ coef,
                                                     const T* __restrict__ theta,
                                                     const T* __restrict__ f, int64_t fcs, Geom gf,
                                                     T* __restrict__ fcoarse, Geom gc,
                                                     const double* __restrict__ wP, LowRankRhs lr) {
  constexpr int S = DIM == 2 ? 9 : 27;
  const int nc = gc.n;
  const int64_t total = int64_t(nc) * nc * (DIM == 3 ? nc : 1);
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= total) return;
  const int c = blockIdx.y;
  int J1, J2, J3;
  unflatten<DIM>(gid, nc, J1, J2, J3);
  const T* th = theta + int64_t(c) * gf.Np;
  const T* fc = f ? f + int64_t(c) * fcs : nullptr;
  const int64_t iJ = pidx(gc, J1, J2, J3);
  T acc = T(0);
#pragma unroll
  for (int t1 = 0; t1 < S; ++t1) {
    const int ex = t1 % 3 - 1, ey = (t1 / 3) % 3 - 1, ez = DIM == 3 ? t1 / 9 - 1 : 0;
    const int64_t ii = pidx(gf, 2 * J1 + ex, 2 * J2 + ey, DIM == 3 ? 2 * J3 + ez : 0);
    T r = fc ? fc[ii] : T(0);
#pragma unroll
    for (int t = 0; t < S; ++t) {
      const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = DIM == 3 ? t / 9 - 1 : 0;
      const int nz = (dx != 0) + (dy != 0) + (dz != 0);
      if (CROSS && nz > 1) continue;
      r -= stencil_entry<T, DIM>(coef, gf, t, ii) * th[ii + poff(gf, dx, dy, dz)];
    }
    const T w = USERP ? T(wP[int64_t(t1) * gc.Np + iJ]) : T(multilinear(ex, ey, ez));
    acc += w * r;
  }
  fcoarse[int64_t(c) * gc.Np + iJ] = T(double(acc) - lowrank_rhs(lr, c, iJ));
}

// Two-stage restriction (used in 3D): r = f - A theta at every fine site,
// then f_{l-1}(J) = sum_delta w_J(delta) r(2J + delta).
template <typename T, int DIM, bool CROSS>
__global__ __launch_bounds__(kBlock) void k_residual(const T* __restrict__ coef,
                                                     const T* __restrict__ theta,
                                                     const T* __restrict__ f, int64_t fcs, Geom g,
                                                     int64_t N, T* __restrict__ r, int cpb,
                                                     int nchains) {
  constexpr int S = DIM == 2 ? 9 : 27;
  constexpr int NS = CROSS ? 2 * DIM + 1 : S;  // stencil entries used
  const int64_t lin = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (lin >= N) return;
  int i1, i2, i3;
  unflatten<DIM>(lin, g.n, i1, i2, i3);
  const int64_t ii = pidx(g, i1, i2, i3);
  T cf[NS];
  int b = 0;
#pragma unroll
  for (int t = 0; t < S; ++t) {
    const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = DIM == 3 ? t / 9 - 1 : 0;
    const int nz = (dx != 0) + (dy != 0) + (dz != 0);
    if (CROSS && nz > 1) continue;
    cf[b++] = stencil_entry<T, DIM>(coef, g, t, ii);
  }
  const int cb = int(blockIdx.y) * cpb;
  const int ce = min(nchains, cb + cpb);
  // two chains per trip, so the loads of the second overlap the first
#pragma unroll 2
  for (int c = cb; c < ce; ++c) {
    const T* th = theta + int64_t(c) * g.Np;
    T acc = f ? f[int64_t(c) * fcs + ii] : T(0);
    b = 0;
#pragma unroll
    for (int t = 0; t < S; ++t) {
      const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = DIM == 3 ? t / 9 - 1 : 0;
      const int nz = (dx != 0) + (dy != 0) + (dz != 0);
      if (CROSS && nz > 1) continue;
      acc -= cf[b++] * th[ii + poff(g, dx, dy, dz)];
    }
    r[int64_t(c) * g.Np + ii] = acc;
  }
}

template <typename T, int DIM, bool USERP>
__global__ __launch_bounds__(kBlock) void k_restrict_residual(const T* __restrict__ r, Geom gf,
                                                              T* __restrict__ fcoarse, Geom gc,
                                                              const double* __restrict__ wP,
                                                              LowRankRhs lr, int cpb, int nchains) {
  constexpr int S = DIM == 2 ? 9 : 27;
  const int nc = gc.n;
  const int64_t total = int64_t(nc) * nc * (DIM == 3 ? nc : 1);
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= total) return;
  int J1, J2, J3;
  unflatten<DIM>(gid, nc, J1, J2, J3);
  const int64_t iJ = pidx(gc, J1, J2, J3);
  const int64_t i0 = pidx(gf, 2 * J1, 2 * J2, DIM == 3 ? 2 * J3 : 0);
  // user weights are loaded once for the thread's group of chains
  T wu[USERP ? S : 1];
  if (USERP) {
#pragma unroll
    for (int t1 = 0; t1 < S; ++t1) wu[t1] = T(wP[int64_t(t1) * gc.Np + iJ]);
  }
  const int cb = int(blockIdx.y) * cpb;
  const int ce = min(nchains, cb + cpb);
  const int brow = lowrank_row(lr, iJ);  // the same for every chain
#pragma unroll 2
  for (int c = cb; c < ce; ++c) {
    const T* rc = r + int64_t(c) * gf.Np;
    T acc = T(0);
#pragma unroll
    for (int t1 = 0; t1 < S; ++t1) {
      const int ex = t1 % 3 - 1, ey = (t1 / 3) % 3 - 1, ez = DIM == 3 ? t1 / 9 - 1 : 0;
      const T w = USERP ? wu[t1] : T(multilinear(ex, ey, ez));
      acc += w * rc[i0 + poff(gf, ex, ey, ez)];
    }
    fcoarse[int64_t(c) * gc.Np + iJ] = T(double(acc) - lowrank_rhs_row(lr, c, brow));
  }
}

template <typename T, int DIM, bool USERP>
__global__ __launch_bounds__(kBlock) void k_prolong(T* __restrict__ theta, Geom gf,
                                                    const T* __restrict__ psi, Geom gc,
                                                    const double* __restrict__ wP, int cpb,
                                                    int nchains) {
  constexpr int NT = DIM == 3 ? 8 : 4;  // coarse terms per fine site
  const int nf = gf.n;
  const int64_t total = int64_t(nf) * nf * (DIM == 3 ? nf : 1);
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= total) return;
  int i[3];
  unflatten<DIM>(gid, nf, i[0], i[1], i[2]);
  // per axis the covering coarse nodes J0 = i >> 1 (offset i & 1) and, for
  // odd i, J1 = (i + 1) >> 1 (offset -1); for even i J1 = J0 with weight 0,
  // so every site sums the same terms in the same order.  Nodes and weights
  // are formed once for the thread's group of chains.
  int J[3][2], D[3][2];
  T h[3][2];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int ik = k < DIM ? i[k] : 0, odd = ik & 1;
    J[k][0] = ik >> 1;
    J[k][1] = (ik + 1) >> 1;
    D[k][0] = odd;
    D[k][1] = -1;
    h[k][0] = odd ? T(0.5) : T(1);
    h[k][1] = odd ? T(0.5) : T(0);
  }
  int64_t jc[NT];
  T w[NT];
  int e = 0;
#pragma unroll
  for (int a3 = 0; a3 < (DIM == 3 ? 2 : 1); ++a3)
#pragma unroll
    for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
      for (int a1 = 0; a1 < 2; ++a1, ++e) {
        jc[e] = pidx(gc, J[0][a1], J[1][a2], J[2][a3]);
        if (USERP) {
          const bool on = (a1 == 0 || (i[0] & 1)) && (a2 == 0 || (i[1] & 1)) &&
                          (DIM == 2 || a3 == 0 || (i[2] & 1));
          const int t = (D[0][a1] + 1) + 3 * (D[1][a2] + 1) + (DIM == 3 ? 9 * (D[2][a3] + 1) : 0);
          w[e] = on ? T(wP[int64_t(t) * gc.Np + jc[e]]) : T(0);
        } else {
          w[e] = h[0][a1] * h[1][a2] * (DIM == 3 ? h[2][a3] : T(1));
        }
      }
  const int64_t ii = pidx(gf, i[0], i[1], i[2]);
  const int cb = int(blockIdx.y) * cpb;
  const int ce = min(nchains, cb + cpb);
  // two chains per trip, so the loads of the second overlap the first
#pragma unroll 2
  for (int c = cb; c < ce; ++c) {
    const T* ps = psi + int64_t(c) * gc.Np;
    T v[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) v[k] = ps[jc[k]];
    T s = w[0] * v[0];
#pragma unroll
    for (int k = 1; k < NT; ++k) s += w[k] * v[k];
    theta[int64_t(c) * gf.Np + ii] += s;
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// theta_0 = K f_0 + U^{-1} z: one wavefront per row, lanes split the row
// (K and U^{-1} row-major, so a wavefront reads contiguous memory).
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_coarsest(const double* __restrict__ K,
                                                     const double* __restrict__ Uinv,
                                                     const T* __restrict__ f0, int64_t fcs,
                                                     T* __restrict__ theta0, Geom g, int N0,
                                                     const int64_t* __restrict__ mcur,
                                                     uint32_t seed, uint32_t chain0, uint32_t word) {
  extern __shared__ double sh[];
  double* fv = sh;
  double* zv = sh + N0;
  const int c = blockIdx.y;
  const uint32_t m = uint32_t(*mcur);
  for (int k = threadIdx.x; k < N0; k += blockDim.x) {
    int i1, i2, i3;
    unflatten<DIM>(k, g.n, i1, i2, i3);
    fv[k] = f0 ? double(f0[int64_t(c) * fcs + pidx(g, i1, i2, i3)]) : 0.0;
  }
  for (int p = threadIdx.x; 2 * p < N0; p += blockDim.x) {
    const Block4 blk = philox10(uint32_t(p), word, m, 2u, seed, chain0 + c);
    double z0, z1;
    Gauss<double>::pair(blk, z0, z1);
    zv[2 * p] = z0;
    if (2 * p + 1 < N0) zv[2 * p + 1] = z1;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int r = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (r >= N0) return;
  double s = 0.0;
  for (int k = lane; k < N0; k += 64) {
    s += K[int64_t(r) * N0 + k] * fv[k];
    if (k >= r) s += Uinv[int64_t(r) * N0 + k] * zv[k];
  }
  s = wave_sum(s);
  if (lane == 0) {
    int i1, i2, i3;
    unflatten<DIM>(r, g.n, i1, i2, i3);
    theta0[int64_t(c) * g.Np + pidx(g, i1, i2, i3)] = T(s);
  }
}

// Low-rank smoother (Alg. 3), first step, one block per chain, one thread
// per observation j: xi_j = Gamma_j^{-1/2} zeta_j and t_j = (B^T theta)_j -
// Gamma_j xi_j.  The correction theta' = theta* - G B^T theta* of the sweep
// output theta* = theta + C xi (C = M^{-1} B, G = C S^{-1}, S = Gamma + B^T C)
// equals theta - G t, because C - G (S - Gamma) = G Gamma.  With v_out it
// also writes v = Gamma^{-1} B^T theta' = xi + S^{-1} t (B^T G = I - Gamma
// S^{-1}), which feeds the low-rank part of the coarse right-hand side.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_lowrank_prep(
    const T* __restrict__ theta, int64_t Np, int beta, const double* __restrict__ gisq,
    const double* __restrict__ gam, const int64_t* __restrict__ bptr,
    const int32_t* __restrict__ bidx, const double* __restrict__ bval,
    const double* __restrict__ SinvT, double* __restrict__ t_out, double* __restrict__ v_out,
    uint32_t word, const int64_t* __restrict__ mcur, uint32_t seed, uint32_t chain0) {
  extern __shared__ double sh[];
  double* xi = sh;              // [beta]
  double* tv = sh + beta;       // [beta]
  double* prod = sh + 2 * beta; // [nnz] weighted site values, then [4][beta] partial sums
  const int c = blockIdx.x;
  const T* th = theta + int64_t(c) * Np;
  const int64_t nnz = bptr[beta];
  // every entry of B^T theta at once: one load chain per entry, no serial
  // walk; four entries per thread are in flight together (branch-free loads
  // of a clamped entry, masked stores)
  for (int64_t e0 = 0; e0 < nnz; e0 += 4 * int64_t(blockDim.x)) {
    double pv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t e = min(e0 + threadIdx.x + int64_t(u) * blockDim.x, nnz - 1);
      pv[u] = bval[e] * double(th[bidx[e]]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t e = e0 + threadIdx.x + int64_t(u) * blockDim.x;
      if (e < nnz) prod[e] = pv[u];
    }
  }
  const uint32_t m = uint32_t(*mcur);
  for (int p = threadIdx.x; 2 * p < beta; p += blockDim.x) {
    const Block4 blk = philox10(uint32_t(p), word, m, 1u, seed, chain0 + c);
    double z0, z1;
    Gauss<double>::pair(blk, z0, z1);
    xi[2 * p] = z0 * gisq[2 * p];
    if (2 * p + 1 < beta) xi[2 * p + 1] = z1 * gisq[2 * p + 1];
  }
  __syncthreads();
  for (int j = threadIdx.x; j < beta; j += blockDim.x) {
    double w = 0.0;
    for (int64_t e = bptr[j]; e < bptr[j + 1]; ++e) w += prod[e];
    const double t = w - gam[j] * xi[j];
    tv[j] = t;
    t_out[int64_t(c) * beta + j] = t;
  }
  if (v_out == nullptr) return;
  __syncthreads();
  // v = xi + S^{-1} t: four threads per row, each over a quarter of the columns
  double* part = prod;
  const int q = int(threadIdx.x) & 3;
  for (int j = int(threadIdx.x) >> 2; j < beta; j += int(blockDim.x) >> 2) {
    double a = 0.0;
#pragma unroll 8
    for (int k = q; k < beta; k += 4) a += SinvT[int64_t(k) * beta + j] * tv[k];
    part[q * beta + j] = a;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < beta; j += blockDim.x)
    v_out[int64_t(c) * beta + j] = xi[j] + ((part[j] + part[beta + j]) + (part[2 * beta + j] + part[3 * beta + j]));
}

// Second step on the support rows: theta_r -= sum_j G_rj t_j for up to CB
// chains per thread, so each entry of G is read once per chain group; four
// threads share a row, each over a quarter of the columns.
template <typename T, int CB>
__global__ __launch_bounds__(kBlock) void k_lowrank_apply(T* __restrict__ theta, int64_t Np,
                                                          int beta, int nsupp,
                                                          const int32_t* __restrict__ supp,
                                                          const double* __restrict__ GT,
                                                          const double* __restrict__ t,
                                                          int nchains) {
  extern __shared__ double sh[];  // [CB][beta] t of the chain group, then [4][CB][64] partials
  double* red = sh + CB * beta;
  const int c0 = blockIdx.y * CB;
  const int nc = min(CB, nchains - c0);
  for (int e = threadIdx.x; e < CB * beta; e += blockDim.x) {
    const int cc = e / beta, j = e % beta;
    sh[e] = cc < nc ? t[int64_t(c0 + cc) * beta + j] : 0.0;
  }
  __syncthreads();
  const int lr = int(threadIdx.x) & 63, q = int(threadIdx.x) >> 6;  // row in block, quarter
  const int r = blockIdx.x * 64 + lr;
  double acc[CB];
#pragma unroll
  for (int cc = 0; cc < CB; ++cc) acc[cc] = 0.0;
  if (r < nsupp) {
#pragma unroll 4
    for (int j = q; j < beta; j += 4) {
      const double g = GT[int64_t(j) * nsupp + r];
#pragma unroll
      for (int cc = 0; cc < CB; ++cc) acc[cc] += g * sh[cc * beta + j];
    }
  }
#pragma unroll
  for (int cc = 0; cc < CB; ++cc) red[(q * CB + cc) * 64 + lr] = acc[cc];
  __syncthreads();
  if (q != 0 || r >= nsupp) return;
  const int64_t at = supp[r];
#pragma unroll
  for (int cc = 0; cc < CB; ++cc) {
    if (cc >= nc) break;
    const double d = (red[cc * 64 + lr] + red[(CB + cc) * 64 + lr]) +
                     (red[(2 * CB + cc) * 64 + lr] + red[(3 * CB + cc) * 64 + lr]);
    T* th = theta + int64_t(c0 + cc) * Np;
    th[at] = T(double(th[at]) - d);
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill_zero(T* __restrict__ p, int64_t count) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) p[i] = T(0);
}

// Per chain and block, the sum of F_i theta_i over the block's range of
// sites (in site order per thread, then by wavefront and lane in a fixed
// tree) into partial[chain][b].  Block (b, y) takes chains 8 y .. 8 y + 7
// and loads the weights of KB sites per thread once for all of them; a
// site with F_i = 0 reads offset 0 of the field (padding, zero) instead of
// theta_i, so that a QoI supported on part of the domain reads only that
// part of the states.
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_qoi_partial(const T* __restrict__ theta, Geom g,
                                                        int64_t N, const double* __restrict__ F,
                                                        double* __restrict__ partial, int nb,
                                                        int nchains) {
  constexpr int KB = 4, CG = kQoiChains, NW = kBlock / 64;
  __shared__ double sh[NW][CG];
  const int b = blockIdx.x, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c0 = int(blockIdx.y) * CG;
  const int64_t chunk = (N + nb - 1) / nb;
  const int64_t lo = int64_t(b) * chunk, hi = lo + chunk < N ? lo + chunk : N;
  const int n = g.n;
  double acc[CG];
#pragma unroll
  for (int cc = 0; cc < CG; ++cc) acc[cc] = 0.0;
  for (int64_t l0 = lo + threadIdx.x; l0 < hi; l0 += KB * blockDim.x) {
    double fv[KB];
    int64_t at[KB];
#pragma unroll
    for (int u = 0; u < KB; ++u) {
      const int64_t lin = l0 + int64_t(u) * blockDim.x;
      fv[u] = F[lin < hi ? lin : lo];
      if (lin >= hi) fv[u] = 0.0;
    }
#pragma unroll
    for (int u = 0; u < KB; ++u) {
      const int l32 = int(l0 + int64_t(u) * blockDim.x);  // N < 2^31 (checked at set-up)
      const int i1 = 1 + l32 % n, r = l32 / n;
      const int i2 = 1 + (DIM == 3 ? r % n : r), i3 = DIM == 3 ? 1 + r / n : 0;
      at[u] = fv[u] != 0.0 ? pidx(g, i1, i2, i3) : 0;
    }
    // chains past the last read the last chain again; their sums are not stored
#pragma unroll
    for (int cc = 0; cc < CG; ++cc) {
      const T* th = theta + int64_t(min(c0 + cc, nchains - 1)) * g.Np;
      double tv[KB];
#pragma unroll
      for (int u = 0; u < KB; ++u) tv[u] = double(th[at[u]]);
#pragma unroll
      for (int u = 0; u < KB; ++u) acc[cc] += fv[u] * tv[u];
    }
  }
#pragma unroll
  for (int cc = 0; cc < CG; ++cc) {
    const double v = wave_sum(acc[cc]);
    if (lane == 0) sh[wave][cc] = v;
  }
  __syncthreads();
  if (int(threadIdx.x) < CG && c0 + int(threadIdx.x) < nchains) {
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) v += sh[w][threadIdx.x];
    partial[int64_t(c0 + int(threadIdx.x)) * nb + b] = v;
  }
}

// One block: wavefront w sums the partials of chains w, w + 4, ... in a
// fixed order, then the sample index advances (the last kernel of an
// update, so no other kernel of this update reads it afterwards).
__global__ __launch_bounds__(kBlock) void k_qoi_final(const double* __restrict__ partial, int nb,
                                                      double* __restrict__ qoi,
                                                      int64_t* __restrict__ mcur, int64_t m0,
                                                      int nchains) {
  const int64_t m = *mcur;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int c = wave; c < nchains; c += kBlock / 64) {
    // 8 loads in flight per lane, added in block order
    const double* pc = partial + int64_t(c) * nb;
    double acc = 0.0;
    for (int b0 = lane; b0 < nb; b0 += 8 * 64) {
      double v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) v[k] = b0 + 64 * k < nb ? pc[b0 + 64 * k] : 0.0;
#pragma unroll
      for (int k = 0; k < 8; ++k) acc += v[k];
    }
    const double s = wave_sum(acc);
    if (lane == 0) qoi[(m - m0) * nchains + c] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) *mcur = m + 1;
}

// Copies between the user's unpadded [chain][N] states and the padded
// layout; a thread takes one site for a group of cpb chains, so the site's
// padded index is formed once for the group.
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_unpack(const T* __restrict__ user, T* __restrict__ th,
                                                   Geom g, int64_t N, int cpb, int nchains) {
  const int64_t lin = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (lin >= N) return;
  int i1, i2, i3;
  unflatten<DIM>(lin, g.n, i1, i2, i3);
  const int64_t ii = pidx(g, i1, i2, i3);
  const int cb = int(blockIdx.y) * cpb, ce = min(nchains, cb + cpb);
#pragma unroll 2
  for (int c = cb; c < ce; ++c) th[int64_t(c) * g.Np + ii] = user[int64_t(c) * N + lin];
}

template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_pack(const T* __restrict__ th, T* __restrict__ user,
                                                 Geom g, int64_t N, int cpb, int nchains) {
  const int64_t lin = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (lin >= N) return;
  int i1, i2, i3;
  unflatten<DIM>(lin, g.n, i1, i2, i3);
  const int64_t ii = pidx(g, i1, i2, i3);
  const int cb = int(blockIdx.y) * cpb, ce = min(nchains, cb + cpb);
#pragma unroll 2
  for (int c = cb; c < ce; ++c) user[int64_t(c) * N + lin] = th[int64_t(c) * g.Np + ii];
}

template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_unpack_rhs(const double* __restrict__ user,
                                                       T* __restrict__ f, Geom g, int64_t N) {
  const int64_t lin = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (lin >= N) return;
  int i1, i2, i3;
  unflatten<DIM>(lin, g.n, i1, i2, i3);
  f[pidx(g, i1, i2, i3)] = T(user[lin]);
}

__global__ void k_set_m(int64_t* mcur, int64_t value) { *mcur = value; }
__global__ void k_advance_m(int64_t* mcur) { *mcur += 1; }

inline unsigned blocks_for(int64_t count) { return unsigned((count + kBlock - 1) / kBlock); }

}  // namespace

#define MGMC_DISPATCH(L, ...)  \
  do {                          \
    if ((L).fp32) {             \
      using T = float;          \
      if ((L).dim == 2) {       \
        constexpr int DIM = 2;  \
        __VA_ARGS__;            \
      } else {                  \
        constexpr int DIM = 3;  \
        __VA_ARGS__;            \
      }                         \
    } else {                    \
      using T = double;         \
      if ((L).dim == 2) {       \
        constexpr int DIM = 2;  \
        __VA_ARGS__;            \
      } else {                  \
        constexpr int DIM = 3;  \
        __VA_ARGS__;            \
      }                         \
    }                           \
  } while (0)

hipError_t launch_sweep_colour(const Launch& L, const DevLevel& lv, void* theta, const void* f,
                               int64_t fcs, uint32_t word, int colour) {
  if (L.mcur == nullptr) return hipErrorInvalidValue;
  const int n = lv.g.n;
  auto ext = [n](int p) { return p ? (n + 1) / 2 : (n - 1) / 2; };
  const int m1 = ext(colour & 1), m2 = ext((colour >> 1) & 1);
  const int m3 = L.dim == 3 ? ext((colour >> 2) & 1) : 1;
  const int64_t total = int64_t((m1 + 1) / 2) * m2 * m3;
  if (total == 0) return hipSuccess;
  const int cpb = chain_group(blocks_for(total), L.nchains, L.cpb_force);
  dim3 grid(blocks_for(total), unsigned((L.nchains + cpb - 1) / cpb));
  MGMC_DISPATCH(L, {
    if (lv.cross)
      k_sweep<T, DIM, true><<<grid, kBlock, 0, L.stream>>>(
          (const T*)lv.coef, (const T*)lv.invd, (const T*)lv.isqd, (T*)theta, (const T*)f, fcs,
          lv.g, colour, word, L.mcur, L.seed, L.chain0, cpb, L.nchains, T(L.omega));
    else
      k_sweep<T, DIM, false><<<grid, kBlock, 0, L.stream>>>(
          (const T*)lv.coef, (const T*)lv.invd, (const T*)lv.isqd, (T*)theta, (const T*)f, fcs,
          lv.g, colour, word, L.mcur, L.seed, L.chain0, cpb, L.nchains, T(L.omega));
  });
  return hipGetLastError();
}

hipError_t launch_sweep_parity3d(const Launch& L, const DevLevel& lv, void* theta, const void* f,
                                  int64_t fcs, uint32_t word, int parity) {
  if (L.mcur == nullptr || L.dim != 3 || !lv.cross) return hipErrorInvalidValue;
  const int n = lv.g.n;
  const int64_t total = int64_t(((n + 1) / 2 + 1) / 2) * n * n;
  const int64_t blocks = blocks_for(total);
  const int cpb = chain_group(blocks, L.nchains, L.cpb_force);
  dim3 grid(unsigned(blocks), unsigned((L.nchains + cpb - 1) / cpb));
  if (L.fp32)
    k_sweep_parity3d<float><<<grid, kBlock, 0, L.stream>>>((const float*)lv.coef, (const float*)lv.invd, (const float*)lv.isqd, (float*)theta, (const float*)f, fcs, lv.g, parity, word, L.mcur, L.seed, L.chain0, cpb, L.nchains, float(L.omega));
  else
    k_sweep_parity3d<double><<<grid, kBlock, 0, L.stream>>>((const double*)lv.coef, (const double*)lv.invd, (const double*)lv.isqd, (double*)theta, (const double*)f, fcs, lv.g, parity, word, L.mcur, L.seed, L.chain0, cpb, L.nchains, L.omega);
  return hipGetLastError();
}

hipError_t launch_restrict(const Launch& L, const DevLevel& fine, const void* theta,
                           const DevLevel& coarse, const void* f, int64_t fcs,
                           const LowRankRhs& lr) {
  dim3 grid(blocks_for(coarse.N), L.nchains);
  MGMC_DISPATCH(L, {
    const T* cf = (const T*)fine.coef;
    const T* th = (const T*)theta;
    T* out = (T*)coarse.f;
    if (fine.wP) {
      if (fine.cross)
        k_restrict<T, DIM, true, true><<<grid, kBlock, 0, L.stream>>>(cf, th, (const T*)f, fcs, fine.g, out, coarse.g, fine.wP, lr);
      else
        k_restrict<T, DIM, false, true><<<grid, kBlock, 0, L.stream>>>(cf, th, (const T*)f, fcs, fine.g, out, coarse.g, fine.wP, lr);
    } else {
      if (fine.cross)
        k_restrict<T, DIM, true, false><<<grid, kBlock, 0, L.stream>>>(cf, th, (const T*)f, fcs, fine.g, out, coarse.g, nullptr, lr);
      else
        k_restrict<T, DIM, false, false><<<grid, kBlock, 0, L.stream>>>(cf, th, (const T*)f, fcs, fine.g, out, coarse.g, nullptr, lr);
    }
  });
  return hipGetLastError();
}

hipError_t launch_restrict_2stage(const Launch& L, const DevLevel& fine, const void* theta,
                                  void* scratch, const DevLevel& coarse, const void* f,
                                  int64_t fcs, const LowRankRhs& lr) {
  if (scratch == nullptr || scratch == theta) return hipErrorInvalidValue;
  if (L.restrict3d && L.dim == 3 && fine.cross && fine.wP == nullptr)
    return launch_restrict3d_lds(L, fine, theta, coarse, f, fcs, lr);
  const int rcpb = chain_group(blocks_for(fine.N), L.nchains, L.cpb_force);
  // FP32: a group of chains per thread amortises the index arithmetic; FP64
  // moves twice the bytes and runs faster with one chain per thread
  const int ccpb = L.fp32 ? chain_group(blocks_for(coarse.N), L.nchains, L.cpb_force) : 1;
  dim3 g1(blocks_for(fine.N), unsigned((L.nchains + rcpb - 1) / rcpb));
  dim3 g2(blocks_for(coarse.N), unsigned((L.nchains + ccpb - 1) / ccpb));
  MGMC_DISPATCH(L, {
    if (fine.cross)
      k_residual<T, DIM, true><<<g1, kBlock, 0, L.stream>>>((const T*)fine.coef, (const T*)theta, (const T*)f, fcs, fine.g, fine.N, (T*)scratch, rcpb, L.nchains);
    else
      k_residual<T, DIM, false><<<g1, kBlock, 0, L.stream>>>((const T*)fine.coef, (const T*)theta, (const T*)f, fcs, fine.g, fine.N, (T*)scratch, rcpb, L.nchains);
    if (fine.wP)
      k_restrict_residual<T, DIM, true><<<g2, kBlock, 0, L.stream>>>((const T*)scratch, fine.g, (T*)coarse.f, coarse.g, fine.wP, lr, ccpb, L.nchains);
    else
      k_restrict_residual<T, DIM, false><<<g2, kBlock, 0, L.stream>>>((const T*)scratch, fine.g, (T*)coarse.f, coarse.g, nullptr, lr, ccpb, L.nchains);
  });
  return hipGetLastError();
}

hipError_t launch_restrict_residual(const Launch& L, const DevLevel& fine, const void* r,
                                    const DevLevel& coarse, const LowRankRhs& lr) {
  const int ccpb = L.fp32 ? chain_group(blocks_for(coarse.N), L.nchains, L.cpb_force) : 1;
  dim3 g2(blocks_for(coarse.N), unsigned((L.nchains + ccpb - 1) / ccpb));
  MGMC_DISPATCH(L, {
    if (fine.wP)
      k_restrict_residual<T, DIM, true><<<g2, kBlock, 0, L.stream>>>((const T*)r, fine.g, (T*)coarse.f, coarse.g, fine.wP, lr, ccpb, L.nchains);
    else
      k_restrict_residual<T, DIM, false><<<g2, kBlock, 0, L.stream>>>((const T*)r, fine.g, (T*)coarse.f, coarse.g, nullptr, lr, ccpb, L.nchains);
  });
  return hipGetLastError();
}

hipError_t launch_prolong(const Launch& L, const DevLevel& fine, void* theta,
                          const DevLevel& coarse, const void* psi) {
  // FP32: a group of chains per thread (as in the restriction)
  const int cpb = L.fp32 ? chain_group(blocks_for(fine.N), L.nchains, L.cpb_force) : 1;
  dim3 grid(blocks_for(fine.N), unsigned((L.nchains + cpb - 1) / cpb));
  MGMC_DISPATCH(L, {
    if (fine.wP)
      k_prolong<T, DIM, true><<<grid, kBlock, 0, L.stream>>>((T*)theta, fine.g, (const T*)psi, coarse.g, fine.wP, cpb, L.nchains);
    else
      k_prolong<T, DIM, false><<<grid, kBlock, 0, L.stream>>>((T*)theta, fine.g, (const T*)psi, coarse.g, nullptr, cpb, L.nchains);
  });
  return hipGetLastError();
}

hipError_t launch_coarsest(const Launch& L, const DevLevel& lv0, const void* f0, int64_t fcs,
                           void* theta0, const double* K, const double* Uinv, uint32_t word) {
  if (L.mcur == nullptr) return hipErrorInvalidValue;
  const int N0 = int(lv0.N);
  const size_t shmem = size_t(2) * N0 * sizeof(double);
  dim3 grid(unsigned((N0 + 3) / 4), unsigned(L.nchains));
  MGMC_DISPATCH(L, {
    k_coarsest<T, DIM><<<grid, kBlock, shmem, L.stream>>>(K, Uinv, (const T*)f0, fcs, (T*)theta0, lv0.g, N0, L.mcur, L.seed, L.chain0, word);
  });
  return hipGetLastError();
}

typedef double mfma_d4 __attribute__((ext_vector_type(4)));

// Products A T on the matrix cores for the 16 rows r0 .. r0 + 15 of one
// wavefront, with A (nrows x beta) stored by columns, A[r][k] = AT[k * lda + r],
// and T (beta x 16 chains) staged in LDS as sT[beta][16], zero past the last
// chain.  The FP64 16x16x4 MFMA takes A[l % 16][l / 16] and B[l / 16][l % 16]
// from lane l and returns D[l / 16 + 4 v][l % 16] in register v.  A is read
// at clamped (valid) indices without branches: rows past nrows are computed
// but not used, and columns past beta meet zeros of T.  mfma_cols_prefetch
// issues the loads of the first 64 columns early, so they can be in flight
// while T is being formed.
__device__ __forceinline__ void mfma_cols_prefetch(double (&av)[16], const double* __restrict__ AT,
                                                   int64_t lda, int nrows, int beta, int r0) {
  const int lane = threadIdx.x & 63;
  const int rc = min(r0 + (lane & 15), nrows - 1), kk = lane >> 4;
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int k = min(4 * u + kk, beta - 1);
    av[u] = AT[int64_t(k) * lda + rc];
  }
}

__device__ __forceinline__ mfma_d4 mfma_rows_product(const double (&av0)[16],
                                                     const double* __restrict__ AT, int64_t lda,
                                                     int nrows, int beta, int r0,
                                                     const double* __restrict__ sT) {
  const int lane = threadIdx.x & 63;
  const int ri = lane & 15, kk = lane >> 4;
  const int rc = min(r0 + ri, nrows - 1);
  mfma_d4 acc = {0.0, 0.0, 0.0, 0.0};
  // chunks of 64 columns: the 16 loads of a chunk are issued together
  for (int kc = 0; kc < beta; kc += 64) {
    double av[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int k = min(kc + 4 * u + kk, beta - 1);
      av[u] = kc == 0 ? av0[u] : AT[int64_t(k) * lda + rc];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int k = kc + 4 * u + kk;
      const double b = k < beta ? sT[k * 16 + ri] : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], b, acc, 0, 0, 0);
    }
  }
  return acc;
}

// theta_r -= sum_j G_rj t_j for the 64 support rows of row block rb (16 per
// wavefront) and chains c0 .. c0 + 15, G given as GT[beta][nsupp].
template <typename T>
struct MfmaRowsPrefetch {
  double av[16];  // G^T entries of the first 64 columns
  double th[4];   // this lane's theta values at its four result rows
  int si[4];      // and their sites, kept for the stores
};

// The loads that do not depend on t: the first column chunk of G and the
// theta values that lowrank_mfma_rows updates.
template <typename T>
__device__ __forceinline__ void lowrank_mfma_prefetch(MfmaRowsPrefetch<T>& pf,
                                                      const T* __restrict__ theta, int64_t Np,
                                                      int beta, int nsupp,
                                                      const int32_t* __restrict__ supp,
                                                      const double* __restrict__ GT, int c0,
                                                      int nchains, int rb) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r0 = rb * 64 + wave * 16;
  mfma_cols_prefetch(pf.av, GT, nsupp, nsupp, beta, r0);
  const T* th = theta + int64_t(min(c0 + (lane & 15), nchains - 1)) * Np;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int rr = min(r0 + (lane >> 4) + 4 * v, nsupp - 1);
    pf.si[v] = supp[rr];
    pf.th[v] = double(th[pf.si[v]]);
  }
}

template <typename T>
__device__ __forceinline__ void lowrank_mfma_rows(const MfmaRowsPrefetch<T>& pf,
                                                  T* __restrict__ theta, int64_t Np, int beta,
                                                  int nsupp, const int32_t* __restrict__ supp,
                                                  const double* __restrict__ GT,
                                                  const double* __restrict__ sT, int c0,
                                                  int nchains, int rb) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r0 = rb * 64 + wave * 16;
  const mfma_d4 acc = mfma_rows_product(pf.av, GT, nsupp, nsupp, beta, r0, sT);
  const int cc = lane & 15;
  if (c0 + cc >= nchains) return;
  T* th = theta + int64_t(c0 + cc) * Np;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int rr = r0 + (lane >> 4) + 4 * v;
    if (rr < nsupp) th[pf.si[v]] = T(pf.th[v] - acc[v]);
  }
}

// The low-rank correction (Alg. 3) in one launch after a 2D sweep that wrote
// its snapshot of B's sites (bsnap: weight times swept value in
// [nchains][beta][KP] slots, zero padded).  Every block forms
// xi = Gamma^{-1/2} zeta and t = B^T theta* - Gamma xi for its group of up to
// 16 chains from the snapshot, which the correction does not modify, so the
// blocks need no ordering among themselves; each column sum takes its KP
// slots in order with all loads issued together.  Blocks x < nrt then apply
// theta -= G t on their 64 support rows; with v_out, blocks x >= nrt instead
// write 64 rows each of v = xi + S^{-1} t for the coarse right-hand side,
// the product S^{-1} t also on the matrix cores.  The noise and the products
// per entry are those of k_lowrank_prep.
template <typename T, int KP>
__global__ __launch_bounds__(kBlock) void k_lowrank_fused_mfma(
    T* __restrict__ theta, int64_t Np, int beta, int nsupp, const int32_t* __restrict__ supp,
    const double* __restrict__ GT, const double* __restrict__ bsnap, int64_t bslots, const double* __restrict__ gisq,
    const double* __restrict__ gam, const double* __restrict__ SinvT, double* __restrict__ v_out,
    int nrt, uint32_t word, const int64_t* __restrict__ mcur, uint32_t seed, uint32_t chain0,
    int nchains) {
  extern __shared__ double sT[];  // [beta][16] t; with v also [beta][16] xi
  double* sX = sT + beta * 16;
  const int c0 = blockIdx.y * 16;
  const int nc = min(16, nchains - c0);
  const bool vblock = int(blockIdx.x) >= nrt;
  const int rv0 = (int(blockIdx.x) - nrt) * 64 + int(threadIdx.x >> 6) * 16;  // v blocks' rows
  const uint32_t m = uint32_t(*mcur);
  MfmaRowsPrefetch<T> pf;
  if (vblock)
    mfma_cols_prefetch(pf.av, SinvT, beta, beta, beta, rv0);
  else
    lowrank_mfma_prefetch<T>(pf, theta, Np, beta, nsupp, supp, GT, c0, nchains, blockIdx.x);
  lowrank_t_xi<KP>(bsnap, bslots, beta, gisq, gam, word, m, seed, chain0, c0, nc, 16,
                   [&](int j, int cc, double t, double xi) {
                     sT[j * 16 + cc] = t;
                     if (vblock) sX[j * 16 + cc] = xi;
                   });
  __syncthreads();
  if (vblock) {
    const mfma_d4 acc = mfma_rows_product(pf.av, SinvT, beta, beta, beta, rv0, sT);
    const int lane = threadIdx.x & 63, cc = lane & 15;
    if (cc >= nc) return;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int j = rv0 + (lane >> 4) + 4 * v;
      if (j < beta) v_out[int64_t(c0 + cc) * beta + j] = sX[j * 16 + cc] + acc[v];
    }
    return;
  }
  lowrank_mfma_rows<T>(pf, theta, Np, beta, nsupp, supp, GT, sT, c0, nchains, blockIdx.x);
}

// The same product on the matrix cores (lowrank_mfma_rows): a block updates
// 64 support rows x 16 chains, with t of the chain group staged in LDS.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_lowrank_apply_mfma(T* __restrict__ theta, int64_t Np,
                                                               int beta, int nsupp,
                                                               const int32_t* __restrict__ supp,
                                                               const double* __restrict__ GT,
                                                               const double* __restrict__ t,
                                                               int nchains, int ngroups) {
  extern __shared__ double sT[];  // [beta][16], zero past the last chain
  // The chain groups of one row tile run on one XCD one after another, so
  // the tile's rows of G come from memory once and from that XCD's L2 for
  // the other groups: linear block b runs on XCD b % 8, and its place
  // q = b / 8 in that XCD's sequence selects chain group q % ngroups of row
  // tile (q / ngroups) * 8 + b % 8.  Row tiles are padded to a multiple of 8.
  const int b = int(blockIdx.x), q = b / 8;
  const int rb = (q / ngroups) * 8 + b % 8;
  if (rb * 64 >= nsupp) return;  // padding tile: the whole block leaves before any barrier
  const int c0 = (q % ngroups) * 16;
  MfmaRowsPrefetch<T> pf;
  lowrank_mfma_prefetch<T>(pf, theta, Np, beta, nsupp, supp, GT, c0, nchains, rb);
  // staged four entries per thread at a time with branch-free loads
  for (int e0 = 0; e0 < beta * 16; e0 += 4 * int(blockDim.x)) {
    double tv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = min(e0 + int(threadIdx.x) + u * int(blockDim.x), beta * 16 - 1);
      const int j = e >> 4, cc = min(c0 + (e & 15), nchains - 1);
      tv[u] = t[int64_t(cc) * beta + j];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + int(threadIdx.x) + u * int(blockDim.x);
      if (e < beta * 16) sT[e] = c0 + (e & 15) < nchains ? tv[u] : 0.0;
    }
  }
  __syncthreads();
  lowrank_mfma_rows<T>(pf, theta, Np, beta, nsupp, supp, GT, sT, c0, nchains, rb);
}

hipError_t launch_lowrank(const Launch& L, const DevLevel& lv, void* theta, int dir, uint32_t word,
                          int beta, const double* gisq, const double* gam, double* t,
                          double* v_out) {
  if (L.mcur == nullptr || (v_out != nullptr && lv.SinvT == nullptr)) return hipErrorInvalidValue;
  if (lv.bnnz > 8192 - 2 * int64_t(beta) || beta > 2048) return hipErrorInvalidValue;
  const size_t pshm = size_t(std::max<int64_t>(2 * beta + lv.bnnz, 6 * int64_t(beta))) * sizeof(double);
  if (L.fp32)
    k_lowrank_prep<float><<<L.nchains, kBlock, pshm, L.stream>>>((const float*)theta, lv.g.Np, beta, gisq, gam, lv.bptr, lv.bidx, lv.bval, lv.SinvT, t, v_out, word, L.mcur, L.seed, L.chain0);
  else
    k_lowrank_prep<double><<<L.nchains, kBlock, pshm, L.stream>>>((const double*)theta, lv.g.Np, beta, gisq, gam, lv.bptr, lv.bidx, lv.bval, lv.SinvT, t, v_out, word, L.mcur, L.seed, L.chain0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || lv.nsupp[dir] == 0) return e;
  if (L.lowrank_mfma && beta <= 512) {  // LDS: beta x 16 doubles <= 64 KiB
    const size_t mshm = size_t(beta) * 16 * sizeof(double);
    const int64_t nrt8 = (int64_t(lv.nsupp[dir]) + 64 * 8 - 1) / (64 * 8) * 8;  // row tiles, padded
    const int ngroups = (L.nchains + 15) / 16;
    const unsigned mgrid = unsigned(nrt8 * ngroups);
    if (L.fp32)
      k_lowrank_apply_mfma<float><<<mgrid, kBlock, mshm, L.stream>>>((float*)theta, lv.g.Np, beta, lv.nsupp[dir], lv.supp[dir], lv.GT[dir], t, L.nchains, ngroups);
    else
      k_lowrank_apply_mfma<double><<<mgrid, kBlock, mshm, L.stream>>>((double*)theta, lv.g.Np, beta, lv.nsupp[dir], lv.supp[dir], lv.GT[dir], t, L.nchains, ngroups);
    return hipGetLastError();
  }
  // chain groups of 8 share each G entry; LDS holds t of the group and the
  // partial sums (<= 64 KiB)
  const int cb = beta <= 768 ? 8 : 1;
  const size_t ashm = (size_t(cb) * beta + size_t(4) * cb * 64) * sizeof(double);
  dim3 agrid(unsigned((lv.nsupp[dir] + 63) / 64), unsigned((L.nchains + cb - 1) / cb));
#define MGMC_LR_APPLY(T, CB)                                                                      \
  k_lowrank_apply<T, CB><<<agrid, kBlock, ashm, L.stream>>>((T*)theta, lv.g.Np, beta, lv.nsupp[dir], \
                                                           lv.supp[dir], lv.GT[dir], t, L.nchains)
  if (L.fp32) {
    if (cb == 8) MGMC_LR_APPLY(float, 8); else MGMC_LR_APPLY(float, 1);
  } else {
    if (cb == 8) MGMC_LR_APPLY(double, 8); else MGMC_LR_APPLY(double, 1);
  }
#undef MGMC_LR_APPLY
  return hipGetLastError();
}

hipError_t launch_lowrank_fused(const Launch& L, const DevLevel& lv, void* theta, int dir,
                                uint32_t word, int beta, const double* gisq, const double* gam,
                                double* v_out) {
  if (L.mcur == nullptr || lv.bsnap == nullptr || beta < 1 || beta > 128) return hipErrorInvalidValue;
  if (lv.bslots != int64_t(beta) * lv.bkp) return hipErrorInvalidValue;
  if (v_out != nullptr && lv.SinvT == nullptr) return hipErrorInvalidValue;
  const int nsupp = lv.nsupp[dir];
  const int nrt = (nsupp + 63) / 64;             // blocks of 64 support rows
  const int nvb = v_out ? (beta + 63) / 64 : 0;  // blocks of 64 rows of v
  if (nrt + nvb == 0) return hipSuccess;
  // LDS: t of 16 chains, with v also their xi (<= 32 KiB for beta <= 128)
  const size_t shm = size_t(beta) * 16 * (v_out ? 2 : 1) * sizeof(double);
  dim3 grid(unsigned(nrt + nvb), unsigned((L.nchains + 15) / 16));
#define MGMC_LR_FUSED(T, KP)                                                                      \
  k_lowrank_fused_mfma<T, KP><<<grid, kBlock, shm, L.stream>>>(                                   \
      (T*)theta, lv.g.Np, beta, nsupp, lv.supp[dir], lv.GT[dir], lv.bsnap, lv.bslots,             \
      gisq, gam, lv.SinvT, v_out, nrt, word, L.mcur, L.seed, L.chain0, L.nchains)
#define MGMC_LR_FUSED_KP(T)                  \
  do {                                       \
    if (lv.bkp == 8) MGMC_LR_FUSED(T, 8);    \
    else if (lv.bkp == 9) MGMC_LR_FUSED(T, 9);   \
    else if (lv.bkp == 12) MGMC_LR_FUSED(T, 12); \
    else if (lv.bkp == 16) MGMC_LR_FUSED(T, 16); \
    else if (lv.bkp == 32) MGMC_LR_FUSED(T, 32); \
    else return hipErrorInvalidValue;        \
  } while (0)
  if (L.fp32)
    MGMC_LR_FUSED_KP(float);
  else
    MGMC_LR_FUSED_KP(double);
#undef MGMC_LR_FUSED_KP
#undef MGMC_LR_FUSED
  return hipGetLastError();
}

hipError_t launch_fill_zero(const Launch& L, void* p, int64_t count) {
  if (count == 0) return hipSuccess;
  if (L.fp32)
    k_fill_zero<float><<<blocks_for(count), kBlock, 0, L.stream>>>((float*)p, count);
  else
    k_fill_zero<double><<<blocks_for(count), kBlock, 0, L.stream>>>((double*)p, count);
  return hipGetLastError();
}

hipError_t launch_qoi(const Launch& L, const DevLevel& fine, const void* theta, const double* F,
                      double* partial, int nb, double* qoi, int64_t m0) {
  if (L.mcur == nullptr || nb < 1) return hipErrorInvalidValue;
  dim3 grid(nb, (L.nchains + kQoiChains - 1) / kQoiChains);
  MGMC_DISPATCH(L, {
    k_qoi_partial<T, DIM><<<grid, kBlock, 0, L.stream>>>((const T*)theta, fine.g, fine.N, F, partial,
                                                         nb, L.nchains);
  });
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_qoi_final<<<1, kBlock, 0, L.stream>>>(partial, nb, qoi, const_cast<int64_t*>(L.mcur), m0,
                                           L.nchains);
  return hipGetLastError();
}

// chain groups in FP32 (as in the prolongation), one chain per thread in FP64
hipError_t launch_unpack(const Launch& L, const DevLevel& lv, const void* user, void* theta) {
  const int cpb = L.fp32 ? chain_group(blocks_for(lv.N), L.nchains, L.cpb_force) : 1;
  dim3 grid(blocks_for(lv.N), unsigned((L.nchains + cpb - 1) / cpb));
  MGMC_DISPATCH(L, { k_unpack<T, DIM><<<grid, kBlock, 0, L.stream>>>((const T*)user, (T*)theta, lv.g, lv.N, cpb, L.nchains); });
  return hipGetLastError();
}

hipError_t launch_pack(const Launch& L, const DevLevel& lv, const void* theta, void* user) {
  const int cpb = L.fp32 ? chain_group(blocks_for(lv.N), L.nchains, L.cpb_force) : 1;
  dim3 grid(blocks_for(lv.N), unsigned((L.nchains + cpb - 1) / cpb));
  MGMC_DISPATCH(L, { k_pack<T, DIM><<<grid, kBlock, 0, L.stream>>>((const T*)theta, (T*)user, lv.g, lv.N, cpb, L.nchains); });
  return hipGetLastError();
}

hipError_t launch_unpack_rhs(const Launch& L, const DevLevel& lv, const double* user, void* f) {
  MGMC_DISPATCH(L, { k_unpack_rhs<T, DIM><<<blocks_for(lv.N), kBlock, 0, L.stream>>>(user, (T*)f, lv.g, lv.N); });
  return hipGetLastError();
}

hipError_t launch_set_m(hipStream_t s, int64_t* mcur, int64_t value) {
  k_set_m<<<1, 1, 0, s>>>(mcur, value);
  return hipGetLastError();
}

hipError_t launch_advance_m(hipStream_t s, int64_t* mcur) {
  k_advance_m<<<1, 1, 0, s>>>(mcur);
  return hipGetLastError();
}

}  // namespace mgmc
