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
#include <type_traits>

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


// ---------------------------------------------------------------------------
// One-launch 3D sweep on the 7-point finest level, marching in z.
//
// A random Gauss-Seidel sweep on a 7-point level is two parity passes (sites
// of one parity sum never couple).  A block owns a TX x TY column of the x-y
// plane over a chunk of planes [za, zb) and marches up through it: at step s
// it runs the first pass at plane s and the second pass at plane s - 1, which
// is the order of the two global passes at every site (the first pass at s
// reads second-parity values at s - 1 before the second pass changes them;
// the second pass at s - 1 reads the first pass's results at s - 2, s - 1 and
// s).  Plane s is staged in LDS for the in-plane neighbours, with a halo of
// two sites in x and y: the first pass also updates the ring of one site
// around the tile (recomputed identically by neighbouring blocks, the noise
// being counter-based), so the second pass on the tile sees final values;
// the chunk likewise starts one plane early.  Each thread owns a segment of
// four sites in x (two Philox pairs, one per x parity, exactly the pairs of
// the parity-pass kernel) and keeps the values of planes s-2 .. s+1 of its
// segment, for a group of chains, in registers, so z neighbours never go
// through memory twice.  Out of place: reads theta_in, writes the tile's
// final planes to theta_out.
constexpr int kMTX = 64, kMSX = kMTX / 4 + 2;
constexpr int kMLS = kMTX + 8 + 1;  // LDS row stride (padded)

// Tile height TY: 24 rows with 512 threads (one block per compute unit) or
// 8 rows with 256 threads (two blocks per compute unit hide each other's
// plane loads, at a larger halo share).
template <typename T, int CPB, int kMTY, int kMNT>
__global__ __launch_bounds__(kMNT) void k_sweep3d_march(
    const T* __restrict__ coef, const T* __restrict__ invd, const T* __restrict__ theta_in,
    T* __restrict__ theta_out, const T* __restrict__ f, Geom g, int first_parity, uint32_t word,
    const int64_t* __restrict__ mcur, uint32_t seed, uint32_t chain0, int tiles_x, int tiles_y,
    int zchunk, int nchains) {
  constexpr int kMSY = kMTY + 4;
  static_assert(kMSX * kMSY <= kMNT, "segment owners exceed the block");
  __shared__ T lds[2][CPB][kMSY][kMLS];
  const int n = g.n;
  const int tid = threadIdx.x;
  const bool active = tid < kMSX * kMSY;
  const int sx = tid % kMSX, sy = tid / kMSX;
  const int tile = blockIdx.x % (tiles_x * tiles_y), bz = blockIdx.x / (tiles_x * tiles_y);
  const int x0 = 1 + kMTX * (tile % tiles_x), y0 = 1 + kMTY * (tile / tiles_x);
  const int xs = x0 - 4 + 4 * sx;       // first site of the segment (1 mod 4)
  const int y = y0 - 2 + (active ? sy : 0);
  const int q = (xs - 1) >> 2;          // segment index
  const int za = 1 + zchunk * bz, zb = min(n + 1, za + zchunk);
  const int c0 = int(blockIdx.y) * CPB;
  const int nc = min(CPB, nchains - c0);
  const uint32_t m = uint32_t(*mcur);
  const int64_t plane = int64_t(g.px) * g.py;
  const bool row_ring = active && y >= y0 - 1 && y <= y0 + kMTY && y >= 1 && y <= n;
  const bool row_tile = active && y >= y0 && y < y0 + kMTY && y <= n;
  // global index of site j of the segment in plane z (padding for positions
  // outside the field: it reads zero and is never written)
  auto gidx = [&](int j, int yy, int z) -> int64_t {
    const int x = xs + j;
    const bool ok = active && x >= 0 && x <= n + 1 && yy >= 0 && yy <= n + 1 && z >= 0 && z <= n + 1;
    return ok ? pidx(g, x, yy, z) : 0;
  };
  auto in_ring = [&](int j) { const int x = xs + j; return row_ring && x >= x0 - 1 && x <= x0 + kMTX && x >= 1 && x <= n; };
  auto in_tile = [&](int j) { const int x = xs + j; return row_tile && x >= x0 && x < x0 + kMTX && x <= n; };
  // per chain, the segment's values in planes s-2 .. s+1 (slot p & 3); every
  // slot index below is a compile-time constant, so the arrays stay in registers
  T v[CPB][4][4];
  // operator of the segment in two planes (slot p & 1): -x entries of sites
  // 0..4, -y and +y, -z and +z entries, inverse diagonal, right-hand side
  T cw[2][5], cs[2][4], cn[2][4], cb[2][4], ct[2][4], ci[2][4], cf[2][4];
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  using I2 = std::integral_constant<int, 2>;
  using I3 = std::integral_constant<int, 3>;
  auto load_plane = [&](auto slot_c, int z) {
    constexpr int slot = decltype(slot_c)::value;
#pragma unroll
    for (int c = 0; c < CPB; ++c) {
      const T* th = theta_in + int64_t(min(c0 + c, nchains - 1)) * g.Np;
#pragma unroll
      for (int j = 0; j < 4; ++j) v[c][slot][j] = th[gidx(j, y, z)];
    }
  };
  auto load_coef = [&](auto set_c, int z) {
    constexpr int k = decltype(set_c)::value;
    const bool zin = z >= 1 && z <= n;
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      const int x = xs + j;
      const bool ok = active && zin && x >= 0 && x <= n + 1 && y >= 0 && y <= n + 1;
      cw[k][j] = coef[int64_t(12) * g.Np + (ok ? pidx(g, x, y, z) : 0)];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t i = zin ? gidx(j, y, z) : 0;
      cs[k][j] = coef[int64_t(10) * g.Np + i];
      cn[k][j] = coef[int64_t(10) * g.Np + (zin ? gidx(j, y + 1, z) : 0)];
      cb[k][j] = coef[int64_t(4) * g.Np + i];
      ct[k][j] = coef[int64_t(4) * g.Np + (i != 0 ? i + plane : 0)];
      ci[k][j] = invd[i];
      cf[k][j] = f ? f[i] : T(0);
    }
  };
  // one pass at plane z over the segment's sites of this pass's x parity
  // (one Philox pair): CUR, LO, HI are the value slots of planes z, z - 1,
  // z + 1, K the operator slot of plane z; the first pass (TILE false) covers
  // the tile and its one-site ring and records its results in LDS buffer K
  // for the second pass; the second (TILE true) covers the tile.
  auto pass = [&](auto cur_c, auto lo_c, auto hi_c, auto k_c, auto tile_c, int z, int parity) {
    constexpr int CUR = decltype(cur_c)::value, LO = decltype(lo_c)::value;
    constexpr int HI = decltype(hi_c)::value, K = decltype(k_c)::value;
    constexpr bool TILE = decltype(tile_c)::value;
    const int xp = (parity + y + z) & 1;  // x parity of this pass's sites
    const int j0 = xp ? 0 : 1;            // sites j0 and j0 + 2 (one Philox pair)
    const bool in0 = TILE ? in_tile(j0) : in_ring(j0);
    const bool in1 = TILE ? in_tile(j0 + 2) : in_ring(j0 + 2);
    if (!in0 && !in1) return;
    const int m1 = xp ? (n + 1) / 2 : (n - 1) / 2;
    const int qx = (m1 + 1) / 2;
    const int m2 = (y & 1) ? (n + 1) / 2 : (n - 1) / 2;
    const uint32_t pair = uint32_t(q) + uint32_t(qx) * (uint32_t((y - 1) >> 1) + uint32_t(m2) * uint32_t((z - 1) >> 1));
    const int colour = xp | ((y & 1) << 1) | ((z & 1) << 2);
    const int col0 = 4 * sx;
#pragma unroll
    for (int c = 0; c < CPB; ++c) {
      if (c >= nc) break;
      const Block4 blk = philox10(pair, word | uint32_t(colour), m, 0u, seed, chain0 + c0 + c);
      T zz[2];
      Gauss<T>::pair(blk, zz[0], zz[1]);
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        // site jj belongs to this pass when jj has the pass's x parity
        if (((jj & 1) == 0) != (xp == 1)) continue;
        const bool inj = (jj >> 1) ? in1 : in0;
        if (!inj) continue;
        const int col = col0 + jj;
        const T xm = jj == 0 ? lds[K][c][sy][col - 1] : v[c][CUR][jj == 0 ? 0 : jj - 1];
        const T xq = jj == 3 ? lds[K][c][sy][col + 1] : v[c][CUR][jj == 3 ? 3 : jj + 1];
        T sum = cf[K][jj];
        sum -= cb[K][jj] * v[c][LO][jj];
        sum -= cs[K][jj] * lds[K][c][sy - 1][col];
        sum -= cw[K][jj] * xm;
        sum -= cw[K][jj + 1] * xq;
        sum -= cn[K][jj] * lds[K][c][sy + 1][col];
        sum -= ct[K][jj] * v[c][HI][jj];
        const T ivd = ci[K][jj];
        const T nv = sum * ivd + zz[jj >> 1] * sqrt(ivd);
        v[c][CUR][jj] = nv;
        if (!TILE) lds[K][c][sy][col] = nv;
      }
    }
  };
  const int sA = za - 1, sE = zb;  // steps s: first pass at s, second at s - 1
  // sA is a multiple of 4 (zchunk is): step sA has phase 0
  load_plane(I3{}, sA - 1);
  load_plane(I0{}, sA);
  load_coef(I0{}, sA);
  auto step = [&](auto phase_c, int s) {
    constexpr int ph = decltype(phase_c)::value;
    using PLO2 = std::integral_constant<int, (ph + 2) & 3>;
    using PLO = std::integral_constant<int, (ph + 3) & 3>;
    using PCUR = std::integral_constant<int, ph>;
    using PHI = std::integral_constant<int, (ph + 1) & 3>;
    using KCUR = std::integral_constant<int, ph & 1>;
    using KPREV = std::integral_constant<int, (ph + 1) & 1>;
    load_plane(PHI{}, s + 1);
    // plane s into LDS (its values so far) for the in-plane neighbours
    if (active) {
#pragma unroll
      for (int c = 0; c < CPB; ++c) {
        if (c >= nc) break;
#pragma unroll
        for (int j = 0; j < 4; ++j) lds[KCUR::value][c][sy][4 * sx + j] = v[c][ph][j];
      }
    }
    __syncthreads();
    if (s >= 1 && s <= n)
      pass(PCUR{}, PLO{}, PHI{}, KCUR{}, std::false_type{}, s, first_parity);
    __syncthreads();
    const int z = s - 1;
    if (z >= za && z < zb && z >= 1 && z <= n) {
      pass(PLO{}, PLO2{}, PCUR{}, KPREV{}, std::true_type{}, z, 1 - first_parity);
#pragma unroll
      for (int c = 0; c < CPB; ++c) {
        if (c >= nc) break;
        T* out = theta_out + int64_t(c0 + c) * g.Np;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (in_tile(j)) out[pidx(g, xs + j, y, z)] = v[c][PLO::value][j];
      }
    }
    __syncthreads();
    load_coef(KPREV{}, s + 1);  // plane s + 1 takes the operator slot of plane s - 1
  };
  for (int s0 = sA; s0 <= sE; s0 += 4) {
    step(I0{}, s0);
    if (s0 + 1 <= sE) step(I1{}, s0 + 1);
    if (s0 + 2 <= sE) step(I2{}, s0 + 2);
    if (s0 + 3 <= sE) step(I3{}, s0 + 3);
  }
}

hipError_t launch_sweep3d_march(const Launch& L, const DevLevel& lv, const void* theta_in,
                                void* theta_out, const void* f, uint32_t word, int backward) {
  if (L.mcur == nullptr || L.dim != 3 || !lv.cross || theta_in == theta_out) return hipErrorInvalidValue;
  const int n = lv.g.n;
  const bool small = L.march3d == 2;
  const int TY = small ? 8 : 24;
  const int tiles_x = (n + kMTX - 1) / kMTX, tiles_y = (n + TY - 1) / TY;
  const int cpb = L.fp32 ? 4 : 1;
  const int groups = (L.nchains + cpb - 1) / cpb;
  // z chunks (a multiple of 4 planes) so that the grid has >= ~1024 blocks
  int zchunk = ((n + 3) / 4) * 4;
  while (zchunk > 16 && int64_t(tiles_x) * tiles_y * groups * ((n + zchunk - 1) / zchunk) < 1024) zchunk -= 4;
  const int nzc = (n + zchunk - 1) / zchunk;
  dim3 grid(unsigned(tiles_x * tiles_y * nzc), unsigned(groups));
  const int first = backward ? 1 : 0;
#define MGMC_MARCH(T, CPB, TYV, NTV)                                                              \
  k_sweep3d_march<T, CPB, TYV, NTV><<<grid, NTV, 0, L.stream>>>(                                  \
      (const T*)lv.coef, (const T*)lv.invd, (const T*)theta_in, (T*)theta_out, (const T*)f, lv.g, \
      first, word, L.mcur, L.seed, L.chain0, tiles_x, tiles_y, zchunk, L.nchains)
  if (L.fp32) {
    if (small) MGMC_MARCH(float, 4, 8, 256); else MGMC_MARCH(float, 4, 24, 512);
  } else {
    if (small) MGMC_MARCH(double, 1, 8, 256); else MGMC_MARCH(double, 1, 24, 512);
  }
#undef MGMC_MARCH
  return hipGetLastError();
}

namespace {

// Residual and full-weighting restriction of a 3D 7-point level in one
// launch (Alg. 1 restriction step, f_{l-1} = P^T (f - A theta) - B_{l-1} v),
// so that the fine residual never goes to memory.  A block owns an 8 x 8 x 4
// tile of coarse nodes.  Per chain it forms, into LDS, the residual on the
// 17 x 17 x 9 fine sites that the tile's restriction stencils cover, from
// theta staged in LDS on those sites plus a ring of one (19 x 19 x 11), and
// each of the first 256 threads sums the 27 weighted residuals of its coarse
// node.  A thread keeps the stencil (and a shared
// right-hand side) of its residual sites in registers for all chains of the
// block.  The sums run in the order of the two-stage form (residual over the
// stencil entries in index order, then the 27 restriction terms in index
// order), so the two forms round alike.
constexpr int kR3X = 8, kR3Y = 8, kR3Z = 4;  // coarse nodes per tile

// kR3NT threads per block: 1024 in single precision (fewer residual sites
// per thread, so more resident wavefronts), 512 in double (a 1024-thread
// block would spill)
template <typename T, int kR3NT>
__global__ __launch_bounds__(kR3NT) void k_restrict3d_lds(
    const T* __restrict__ coef, const T* __restrict__ theta, const T* __restrict__ f, int64_t fcs,
    Geom gf, T* __restrict__ fcoarse, Geom gc, LowRankRhs lr, int tiles_x, int tiles_y,
    int tiles_z, int per_xcd, int cpb, int nchains) {
  constexpr int RX = 2 * kR3X + 1, RY = 2 * kR3Y + 1, RZ = 2 * kR3Z + 1;  // residual region
  constexpr int HX = RX + 2, HY = RY + 2, HZ = RZ + 2;                    // state region
  constexpr int NR = RX * RY * RZ, NH = HX * HY * HZ;
  constexpr int KR = (NR + kR3NT - 1) / kR3NT, KH = (NH + kR3NT - 1) / kR3NT;
  static_assert(kR3X * kR3Y * kR3Z <= kR3NT, "one coarse node per thread");
  __shared__ T sth[NH];
  __shared__ T sr[NR];
  const int n = gf.n, nc = gc.n;
  const int tid = int(threadIdx.x);
  // Each XCD takes a contiguous range of tiles (x fastest, then y, then z),
  // so the neighbouring tiles whose state regions overlap run on one XCD and
  // share its L2: linear block b runs on XCD b % 8 and takes tile
  // (b % 8) * per_xcd + b / 8 (the tile count padded to 8 * per_xcd).
  const int tile = (int(blockIdx.x) % 8) * per_xcd + int(blockIdx.x) / 8;
  if (tile >= tiles_x * tiles_y * tiles_z) return;  // padding: the whole block leaves before any barrier
  const int bx = tile % tiles_x, by = (tile / tiles_x) % tiles_y, bz = tile / (tiles_x * tiles_y);
  const int J0x = bx * kR3X + 1, J0y = by * kR3Y + 1, J0z = bz * kR3Z + 1;
  // origin of the state region: fine node 2 J0 - 2 (the residual region
  // starts one site further, at 2 J0 - 1 >= 1)
  const int h0x = 2 * J0x - 2, h0y = 2 * J0y - 2, h0z = 2 * J0z - 2;
  // The thread's residual sites.  Sites past n belong only to coarse nodes
  // outside the grid: zero stencil, never read.
  // (field offsets fit 32 bits: the launcher checks Np)
  T cf[KR][7], fr[KR];
  int gi[KR];
#pragma unroll
  for (int k = 0; k < KR; ++k) {
    const int s = min(tid + k * kR3NT, NR - 1);
    const int rx = s % RX, ry = (s / RX) % RY, rz = s / (RX * RY);
    const int x = h0x + 1 + rx, y = h0y + 1 + ry, z = h0z + 1 + rz;
    const bool in = x <= n && y <= n && z <= n;
    gi[k] = in ? int(pidx(gf, x, y, z)) : -1;
    const int64_t i = in ? int64_t(gi[k]) : pidx(gf, 1, 1, 1);
    int b = 0;
#pragma unroll
    for (int t = 0; t < 27; ++t) {
      const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
      if ((dx != 0) + (dy != 0) + (dz != 0) > 1) continue;
      cf[k][b++] = in ? stencil_entry<T, 3>(coef, gf, t, i) : T(0);
    }
    fr[k] = (in && f != nullptr && fcs == 0) ? f[i] : T(0);
  }
  // offsets of the thread's state-region loads (positions past the last
  // ghost plane clamped onto it: they feed only residual sites that no
  // coarse node reads)
  int ho[KH];
#pragma unroll
  for (int k = 0; k < KH; ++k) {
    const int s = min(tid + k * kR3NT, NH - 1);
    const int hx = s % HX, hy = (s / HX) % HY, hz = s / (HX * HY);
    ho[k] = int(pidx(gf, min(h0x + hx, n + 1), min(h0y + hy, n + 1), min(h0z + hz, n + 1)));
  }
  // the thread's coarse node (first 256 threads)
  const int cx = tid % kR3X, cy = (tid / kR3X) % kR3Y, cz = tid / (kR3X * kR3Y);
  const int Jx = J0x + cx, Jy = J0y + cy, Jz = J0z + cz;
  const bool jin = tid < kR3X * kR3Y * kR3Z && Jx <= nc && Jy <= nc && Jz <= nc;
  const int64_t iJ = jin ? pidx(gc, Jx, Jy, Jz) : 0;
  const int brow = jin ? lowrank_row(lr, iJ) : -1;  // the same for every chain
  const int rb = (2 * cx + 1) + RX * ((2 * cy + 1) + RY * (2 * cz + 1));
  const int cb = int(blockIdx.y) * cpb;
  const int ce = min(nchains, cb + cpb);
  // The state region of chain c + 1 is loaded into registers while chain c
  // forms its residual, and moved into LDS once chain c no longer reads it.
  T hv[KH];
  auto load = [&](int c) {
    const T* th = theta + int64_t(c) * gf.Np;
#pragma unroll
    for (int k = 0; k < KH; ++k) hv[k] = th[ho[k]];
  };
  auto stage = [&]() {
#pragma unroll
    for (int k = 0; k < KH; ++k)
      if (tid + k * kR3NT < NH) sth[tid + k * kR3NT] = hv[k];
  };
  if (cb < ce) {
    load(cb);
    stage();
  }
  if (cb + 1 < ce) load(cb + 1);
  for (int c = cb; c < ce; ++c) {
    __syncthreads();  // sth holds chain c; the previous chain's restriction has read sr
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      if (tid + k * kR3NT >= NR) continue;
      T acc = fcs == 0 ? fr[k] : ((gi[k] >= 0 && f != nullptr) ? f[int64_t(c) * fcs + gi[k]] : T(0));
      const int s = tid + k * kR3NT;
      const int h = (s % RX + 1) + HX * ((s / RX) % RY + 1 + HY * (s / (RX * RY) + 1));
      acc -= cf[k][0] * sth[h - HX * HY];  // (0, 0, -1)
      acc -= cf[k][1] * sth[h - HX];       // (0, -1, 0)
      acc -= cf[k][2] * sth[h - 1];        // (-1, 0, 0)
      acc -= cf[k][3] * sth[h];            // centre
      acc -= cf[k][4] * sth[h + 1];        // (+1, 0, 0)
      acc -= cf[k][5] * sth[h + HX];       // (0, +1, 0)
      acc -= cf[k][6] * sth[h + HX * HY];  // (0, 0, +1)
      sr[tid + k * kR3NT] = acc;
    }
    __syncthreads();  // sr holds chain c; no thread reads sth until the next barrier
    if (c + 1 < ce) stage();
    if (c + 2 < ce) load(c + 2);
    if (jin) {
      T acc = T(0);
#pragma unroll
      for (int t1 = 0; t1 < 27; ++t1) {
        const int ex = t1 % 3 - 1, ey = (t1 / 3) % 3 - 1, ez = t1 / 9 - 1;
        acc += T(multilinear(ex, ey, ez)) * sr[rb + ex + RX * (ey + RY * ez)];
      }
      fcoarse[int64_t(c) * gc.Np + iJ] = T(double(acc) - lowrank_rhs_row(lr, c, brow));
    }
  }
}

}  // namespace

hipError_t launch_restrict3d_lds(const Launch& L, const DevLevel& fine, const void* theta,
                                 const DevLevel& coarse, const void* f, int64_t fcs,
                                 const LowRankRhs& lr) {
  if (L.dim != 3 || !fine.cross || fine.wP != nullptr || coarse.g.n != (fine.g.n - 1) / 2 ||
      fine.g.Np >= (int64_t(1) << 31))
    return hipErrorInvalidValue;
  const int nc = coarse.g.n;
  const int tiles_x = (nc + kR3X - 1) / kR3X, tiles_y = (nc + kR3Y - 1) / kR3Y,
            tiles_z = (nc + kR3Z - 1) / kR3Z;
  const int64_t tiles = int64_t(tiles_x) * tiles_y * tiles_z;
  // chain groups as the per-site kernels choose them, from the tile count
  const int cpb = chain_group(tiles, L.nchains, L.cpb_force);
  const int per_xcd = int((tiles + 7) / 8);
  dim3 grid(unsigned(8 * per_xcd), unsigned((L.nchains + cpb - 1) / cpb));
  if (L.fp32)
    k_restrict3d_lds<float, 1024><<<grid, 1024, 0, L.stream>>>(
        (const float*)fine.coef, (const float*)theta, (const float*)f, fcs, fine.g,
        (float*)coarse.f, coarse.g, lr, tiles_x, tiles_y, tiles_z, per_xcd, cpb, L.nchains);
  else
    k_restrict3d_lds<double, 512><<<grid, 512, 0, L.stream>>>(
        (const double*)fine.coef, (const double*)theta, (const double*)f, fcs, fine.g,
        (double*)coarse.f, coarse.g, lr, tiles_x, tiles_y, tiles_z, per_xcd, cpb, L.nchains);
  return hipGetLastError();
}

}  // namespace mgmc
