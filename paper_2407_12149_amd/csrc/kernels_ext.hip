// HIP kernels of the wider operators and of the single-level exact sampler.
//
//  * k_sweep_wide: one colour pass of the random Gauss-Seidel / SOR smoother
//    (Alg. 2/3, M = D / omega + L in colour order) on a 2D level with a 5 x 5
//    stencil: the 13-point squared shifted Laplace and its 25-point Galerkin
//    coarse operators (Sec. 5.1.1).  Same-coloured sites, (i_1 mod 3,
//    i_2 mod 3) fixed, are three apart and never couple.  One thread owns one
//    Philox block: the two sites of the colour's sublattice at x-distance 3
//    that share it (pair = (s_1 >> 1) + ceil(m_1 / 2) s_2, slot s_1 & 1, with
//    s_k = (i_k - 1) / 3 the sublattice coordinates and m_1 the sublattice
//    extent along x).
//  * k_residual_wide: r = f - A theta on such a level (the restriction then
//    applies P^T, Alg. 1 restriction step).
//  * k_band_*: the exact sampler theta = mu + U^{-1} z of Sec. 5.1.3 with a
//    banded Cholesky factor At = U^T U (lexicographic order), by blocked back
//    substitution in one workgroup per group of chains.
#include <algorithm>

#include "device_common.h"
#include "device_rng.h"
#include "mgmc_internal.h"

namespace mgmc {

namespace {

constexpr int kS25 = 25;

// Entry t of the 5 x 5 stencil of site i (t = (dx + 2) + 5 (dy + 2)); past
// the centre it is the opposite entry of the neighbour (symmetric operator),
// so only the centre and the lower half come from memory.
template <typename T>
__device__ __forceinline__ T entry25(const T* __restrict__ coef, const Geom& g, int t, int64_t i) {
  if (t <= kS25 / 2) return coef[int64_t(t) * g.Np + i];
  const int dx = t % 5 - 2, dy = t / 5 - 2;
  return coef[int64_t(kS25 - 1 - t) * g.Np + i + dx + int64_t(g.px) * dy];
}

template <typename T>
__device__ __forceinline__ T sor_site_w(T old, T s, T ivd, T isd, T z, T om) {
  return (T(1) - om) * old + om * (s * ivd) + sqrt(om * (T(2) - om)) * isd * z;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_sweep_wide(const T* __restrict__ coef,
                                                       const T* __restrict__ invd,
                                                       T* __restrict__ theta,
                                                       const T* __restrict__ f, int64_t fcs, Geom g,
                                                       int colour, uint32_t word,
                                                       const int64_t* __restrict__ mcur,
                                                       uint32_t seed, uint32_t chain0, int cpb,
                                                       int nchains, T om) {
  const int n = g.n;
  const int p1 = colour % 3, p2 = colour / 3;
  const int first1 = p1 == 0 ? 3 : p1, first2 = p2 == 0 ? 3 : p2;
  const int m1 = first1 <= n ? (n - first1) / 3 + 1 : 0;
  const int m2 = first2 <= n ? (n - first2) / 3 + 1 : 0;
  const int qx = (m1 + 1) / 2;
  const int64_t total = int64_t(qx) * m2;
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= total) return;
  const int q = int(gid % qx), s2 = int(gid / qx);
  const int i1 = first1 + 6 * q, i2 = first2 + 3 * s2;
  const bool two = 2 * q + 1 < m1;
  const uint32_t pair = uint32_t(q) + uint32_t(qx) * uint32_t(s2);
  const uint32_t m = uint32_t(*mcur);
  const int64_t ia = pidx(g, i1, i2, 0);
  // a missing second site (past the row end) reads padding and halo entries,
  // which are zero and inside the field, and is not stored
  T cf[2][kS25 - 1], ivd[2], isd[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int64_t i = ia + 3 * k;
    int b = 0;
#pragma unroll
    for (int t = 0; t < kS25; ++t) {
      if (t == kS25 / 2) continue;
      cf[k][b++] = entry25(coef, g, t, i);
    }
    ivd[k] = invd[i];
    isd[k] = sqrt(ivd[k]);
  }
  const int cb = int(blockIdx.y) * cpb;
  const int ce = min(nchains, cb + cpb);
  for (int c = cb; c < ce; ++c) {
    T* th = theta + int64_t(c) * g.Np;
    T s[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int64_t i = ia + 3 * k;
      s[k] = f ? f[int64_t(c) * fcs + i] : T(0);
      int b = 0;
#pragma unroll
      for (int t = 0; t < kS25; ++t) {
        if (t == kS25 / 2) continue;
        const int dx = t % 5 - 2, dy = t / 5 - 2;
        s[k] -= cf[k][b++] * th[i + dx + int64_t(g.px) * dy];
      }
    }
    const Block4 blk = philox10(pair, word | uint32_t(colour), m, 0u, seed, chain0 + c);
    T z[2];
    Gauss<T>::pair(blk, z[0], z[1]);
    if (om == T(1)) {
      th[ia] = s[0] * ivd[0] + z[0] * isd[0];
      if (two) th[ia + 3] = s[1] * ivd[1] + z[1] * isd[1];
    } else {
      th[ia] = sor_site_w(th[ia], s[0], ivd[0], isd[0], z[0], om);
      if (two) th[ia + 3] = sor_site_w(th[ia + 3], s[1], ivd[1], isd[1], z[1], om);
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_residual_wide(const T* __restrict__ coef,
                                                          const T* __restrict__ theta,
                                                          const T* __restrict__ f, int64_t fcs,
                                                          Geom g, T* __restrict__ r, int nchains) {
  const int n = g.n;
  const int64_t lin = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (lin >= int64_t(n) * n) return;
  const int i1 = 1 + int(lin % n), i2 = 1 + int(lin / n);
  const int64_t ii = pidx(g, i1, i2, 0);
  T cf[kS25];
#pragma unroll
  for (int t = 0; t < kS25; ++t) cf[t] = entry25(coef, g, t, ii);
  for (int c = int(blockIdx.y); c < nchains; c += gridDim.y) {
    const T* th = theta + int64_t(c) * g.Np;
    T acc = f ? f[int64_t(c) * fcs + ii] : T(0);
#pragma unroll
    for (int t = 0; t < kS25; ++t) {
      const int dx = t % 5 - 2, dy = t / 5 - 2;
      acc -= cf[t] * th[ii + dx + int64_t(g.px) * dy];
    }
    r[int64_t(c) * g.Np + ii] = acc;
  }
}

// x[c][i] = z_i: the normals of the exact sample, pair i >> 1, slot i & 1,
// stream tag 2 (as on the coarsest level of a V-cycle).
__global__ __launch_bounds__(kBlock) void k_band_noise(double* __restrict__ x, int64_t N,
                                                       const int64_t* __restrict__ mcur,
                                                       uint32_t seed, uint32_t chain0,
                                                       uint32_t word) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (2 * p >= N) return;
  const int c = blockIdx.y;
  const Block4 blk = philox10(uint32_t(p), word, uint32_t(*mcur), 2u, seed, chain0 + c);
  double z0, z1;
  Gauss<double>::pair(blk, z0, z1);
  x[int64_t(c) * N + 2 * p] = z0;
  if (2 * p + 1 < N) x[int64_t(c) * N + 2 * p + 1] = z1;
}

constexpr int kBandRows = 64;   // rows per block step
constexpr int kBandChains = 4;  // chains per workgroup (one wavefront each on the triangle)

// Back substitution U x = z in place, bottom block first.  For the block of
// rows [r0, r1): the wavefront of each chain solves the triangle (lane k
// holds row r0 + k; the triangle of U is staged in LDS), then all threads
// subtract the block's contribution from the `band` rows above it, reading
// each entry of U once for the workgroup's chains.
__global__ __launch_bounds__(kBlock) void k_band_backsolve(const double* __restrict__ U,
                                                           int64_t N, int64_t W,
                                                           double* __restrict__ x, int nchains) {
  __shared__ double tri[kBandRows][kBandRows + 1];
  __shared__ double xs[kBandChains][kBandRows];
  const int c0 = int(blockIdx.x) * kBandChains;
  const int nc = min(kBandChains, nchains - c0);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t band = W - 1;
  const int64_t nblk = (N + kBandRows - 1) / kBandRows;
  for (int64_t kb = nblk - 1; kb >= 0; --kb) {
    const int64_t r0 = kb * kBandRows;
    const int rows = int(min<int64_t>(kBandRows, N - r0));
    // triangle: tri[a][b] = U(r0 + a, r0 + b), b >= a, zero outside the band
    for (int e = threadIdx.x; e < kBandRows * kBandRows; e += kBlock) {
      const int a = e / kBandRows, b = e % kBandRows;
      double v = 0.0;
      if (a < rows && b < rows && b >= a && b - a <= band) v = U[(r0 + a) * W + (b - a)];
      tri[a][b] = v;
    }
    __syncthreads();
    if (wave < nc) {
      double* xc = x + int64_t(c0 + wave) * N;
      double y = lane < rows ? xc[r0 + lane] : 0.0;
      for (int i = rows - 1; i >= 0; --i) {
        const double xi = __shfl(y / tri[i][i], i, 64);
        if (lane == i) y = xi;
        if (lane < i) y -= tri[lane][i] * xi;
      }
      if (lane < rows) {
        xc[r0 + lane] = y;
        xs[wave][lane] = y;
      }
    }
    __syncthreads();
    // rows j in [max(0, r0 - band), r0) lose sum_b U(j, r0 + b) x_{r0 + b}
    const int64_t j0 = r0 - band > 0 ? r0 - band : 0;
    for (int64_t j = j0 + threadIdx.x; j < r0; j += kBlock) {
      const double* uj = U + j * W;
      const int64_t d0 = r0 - j;  // offset of column r0 in row j
      const int bmax = int(min<int64_t>(rows, band - d0 + 1));
      double acc[kBandChains] = {0.0, 0.0, 0.0, 0.0};
      for (int b = 0; b < bmax; ++b) {
        const double u = uj[d0 + b];
#pragma unroll
        for (int cc = 0; cc < kBandChains; ++cc) acc[cc] += u * xs[cc][b];
      }
      for (int cc = 0; cc < nc; ++cc) x[int64_t(c0 + cc) * N + j] -= acc[cc];
    }
    __syncthreads();
  }
}

template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_band_finish(const double* __restrict__ x,
                                                        const double* __restrict__ mu, int64_t N,
                                                        Geom g, T* __restrict__ theta) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int c = blockIdx.y;
  int i1, i2, i3;
  unflatten<DIM>(i, g.n, i1, i2, i3);
  const double v = x[int64_t(c) * N + i] + (mu ? mu[i] : 0.0);
  theta[int64_t(c) * g.Np + pidx(g, i1, i2, i3)] = T(v);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_broadcast(const T* __restrict__ src, T* __restrict__ dst,
                                                      int64_t Np) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= Np) return;
  dst[int64_t(blockIdx.y) * Np + i] = src ? src[i] : T(0);
}

inline unsigned blocks_of(int64_t count) { return unsigned((count + kBlock - 1) / kBlock); }

}  // namespace

hipError_t launch_broadcast(const Launch& L, const DevLevel& lv, const void* src, void* dst) {
  dim3 grid(blocks_of(lv.g.Np), unsigned(L.nchains));
  if (L.fp32)
    k_broadcast<float><<<grid, kBlock, 0, L.stream>>>((const float*)src, (float*)dst, lv.g.Np);
  else
    k_broadcast<double><<<grid, kBlock, 0, L.stream>>>((const double*)src, (double*)dst, lv.g.Np);
  return hipGetLastError();
}

hipError_t launch_sweep_wide(const Launch& L, const DevLevel& lv, void* theta, const void* f,
                             int64_t fcs, uint32_t word, int colour) {
  if (L.mcur == nullptr || L.dim != 2) return hipErrorInvalidValue;
  const int n = lv.g.n;
  const int p1 = colour % 3, p2 = colour / 3;
  const int f1 = p1 == 0 ? 3 : p1, f2 = p2 == 0 ? 3 : p2;
  const int m1 = f1 <= n ? (n - f1) / 3 + 1 : 0, m2 = f2 <= n ? (n - f2) / 3 + 1 : 0;
  const int64_t total = int64_t((m1 + 1) / 2) * m2;
  if (total == 0) return hipSuccess;
  // chains per block: enough blocks to fill the device, up to 8 chains
  int cpb = std::min(L.nchains, 8);
  while (cpb > 1 && int64_t(blocks_of(total)) * ((L.nchains + cpb - 1) / cpb) < 1024) cpb /= 2;
  dim3 grid(blocks_of(total), unsigned((L.nchains + cpb - 1) / cpb));
  if (L.fp32)
    k_sweep_wide<float><<<grid, kBlock, 0, L.stream>>>((const float*)lv.coef, (const float*)lv.invd, (float*)theta, (const float*)f, fcs, lv.g, colour, word, L.mcur, L.seed, L.chain0, cpb, L.nchains, float(L.omega));
  else
    k_sweep_wide<double><<<grid, kBlock, 0, L.stream>>>((const double*)lv.coef, (const double*)lv.invd, (double*)theta, (const double*)f, fcs, lv.g, colour, word, L.mcur, L.seed, L.chain0, cpb, L.nchains, L.omega);
  return hipGetLastError();
}

hipError_t launch_restrict_wide(const Launch& L, const DevLevel& fine, const void* theta,
                                void* scratch, const DevLevel& coarse, const void* f, int64_t fcs,
                                const LowRankRhs& lr) {
  if (scratch == nullptr || scratch == theta || L.dim != 2) return hipErrorInvalidValue;
  dim3 g1(blocks_of(fine.N), unsigned(std::min(L.nchains, 64)));
  if (L.fp32)
    k_residual_wide<float><<<g1, kBlock, 0, L.stream>>>((const float*)fine.coef, (const float*)theta, (const float*)f, fcs, fine.g, (float*)scratch, L.nchains);
  else
    k_residual_wide<double><<<g1, kBlock, 0, L.stream>>>((const double*)fine.coef, (const double*)theta, (const double*)f, fcs, fine.g, (double*)scratch, L.nchains);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_restrict_residual(L, fine, scratch, coarse, lr);
}

hipError_t launch_band_sample(const Launch& L, const DevLevel& lv, const double* U, int64_t band,
                              const double* mu, double* x, void* theta, uint32_t word) {
  if (L.mcur == nullptr || U == nullptr || x == nullptr) return hipErrorInvalidValue;
  const int64_t N = lv.N;
  dim3 gn(blocks_of((N + 1) / 2), unsigned(L.nchains));
  k_band_noise<<<gn, kBlock, 0, L.stream>>>(x, N, L.mcur, L.seed, L.chain0, word);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned groups = unsigned((L.nchains + kBandChains - 1) / kBandChains);
  k_band_backsolve<<<groups, kBlock, 0, L.stream>>>(U, N, band + 1, x, L.nchains);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  dim3 gf(blocks_of(N), unsigned(L.nchains));
  if (L.dim == 2) {
    if (L.fp32)
      k_band_finish<float, 2><<<gf, kBlock, 0, L.stream>>>(x, mu, N, lv.g, (float*)theta);
    else
      k_band_finish<double, 2><<<gf, kBlock, 0, L.stream>>>(x, mu, N, lv.g, (double*)theta);
  } else {
    if (L.fp32)
      k_band_finish<float, 3><<<gf, kBlock, 0, L.stream>>>(x, mu, N, lv.g, (float*)theta);
    else
      k_band_finish<double, 3><<<gf, kBlock, 0, L.stream>>>(x, mu, N, lv.g, (double*)theta);
  }
  return hipGetLastError();
}

}  // namespace mgmc
