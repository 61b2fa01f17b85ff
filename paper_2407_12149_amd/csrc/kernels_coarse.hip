// The bottom of the V-cycle in one launch: one workgroup per chain runs every
// level from lm down to the coarsest and back up (Alg. 1 restricted to levels
// 0..lm), with the states and right-hand sides of those levels resident in
// LDS.  Below about 63^2 sites per level each step is far too small to fill
// the device, so the separate launches would cost latency only; here the
// workgroup's barriers replace them.
//
// Per level l (2D, Galerkin 9-point), going down: forward colour-ordered
// random Gauss-Seidel sweep(s) (Alg. 2/3), the low-rank correction of Alg. 3
// (theta -= G (B^T theta - Gamma xi)), and the restriction
// f_{l-1} = P^T (f_l - A_l theta_l) - B_{l-1} v; on level 0 the exact sample
// theta_0 = K f_0 + U^{-1} z (Sec. 3.5); going up: theta_l += P theta_{l-1}
// (multilinear, Sec. 3.1), backward sweep(s) and their low-rank correction.
// Noise counters, summation orders and precisions follow the per-level
// kernels, so the chains are the same up to rounding.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.h"
#include "device_rng.h"
#include "mgmc_internal.h"

namespace mgmc {

namespace {

constexpr int kCT = 512;  // threads per workgroup
constexpr int kFwd[4] = {0, 3, 1, 2};

// One colour-ordered sweep of level A on the LDS state th (in place).
template <typename T>
__device__ void cv_sweep(const CoarseLevel& A, T* __restrict__ th, const T* __restrict__ f,
                         uint32_t word, bool backward, uint32_t m, uint32_t seed, uint32_t chain) {
  const Geom g = A.g;
  const int n = g.n;
  const T* __restrict__ coef = (const T*)A.coef;
  const T* __restrict__ invd = (const T*)A.invd;
  const T* __restrict__ isqd = (const T*)A.isqd;
  for (int qc = 0; qc < 4; ++qc) {
    const int colour = kFwd[backward ? 3 - qc : qc];
    const int p1 = colour & 1, p2 = (colour >> 1) & 1;
    const int m1 = p1 ? (n + 1) / 2 : (n - 1) / 2;
    const int m2 = p2 ? (n + 1) / 2 : (n - 1) / 2;
    const int qx = (m1 + 1) / 2;
    for (int gid = threadIdx.x; gid < qx * m2; gid += blockDim.x) {
      const int q = gid % qx, s2 = gid / qx;
      const int i1 = 4 * q + (p1 ? 1 : 2), i2 = 2 * s2 + (p2 ? 1 : 2);
      const uint32_t pair = uint32_t(q) + uint32_t(qx) * uint32_t(s2);
      const Block4 blk = philox10(pair, word | uint32_t(colour), m, 0u, seed, chain);
      T z[2];
      Gauss<T>::pair(blk, z[0], z[1]);
      for (int k = 0; k < 2; ++k) {
        if (k == 1 && 2 * q + 1 >= m1) break;
        const int64_t ia = pidx(g, i1 + 2 * k, i2, 0);
        T s = f[ia];
#pragma unroll
        for (int t = 0; t < 9; ++t) {
          if (t == 4) continue;
          s -= stencil_entry<T, 2>(coef, g, t, ia) * th[ia + poff(g, t % 3 - 1, t / 3 - 1, 0)];
        }
        th[ia] = s * invd[ia] + z[k] * isqd[ia];
      }
    }
    __syncthreads();
  }
}

// Low-rank correction of Alg. 3 on level A after a sweep in direction dir:
// xi = Gamma^{-1/2} zeta, t = B^T theta - Gamma xi, theta -= G t on the
// support rows; with want_v also v = xi + S^{-1} t (Gamma^{-1} B^T theta').
// Every global load is issued with many others in flight (one workgroup has
// to hide the latency on its own): the entries of B^T theta at once, 16
// threads per row of S^{-1}, and rows of G in chunks of 16 unrolled loads.
template <typename T>
__device__ void cv_lowrank(const CoarseLevel& A, const CoarseCommon& C, T* __restrict__ th, int dir,
                           uint32_t word, bool want_v, double* __restrict__ xi,
                           double* __restrict__ tv, double* __restrict__ vv,
                           double* __restrict__ scr, uint32_t m, uint32_t chain) {
  const int beta = C.beta;
  const int64_t nnz = A.bptr[beta];
  for (int64_t e = threadIdx.x; e < nnz; e += blockDim.x) scr[e] = A.bval[e] * double(th[A.bidx[e]]);
  for (int p = threadIdx.x; 2 * p < beta; p += blockDim.x) {
    const Block4 blk = philox10(uint32_t(p), word, m, 1u, C.seed, chain);
    double z0, z1;
    Gauss<double>::pair(blk, z0, z1);
    xi[2 * p] = z0 * C.gisq[2 * p];
    if (2 * p + 1 < beta) xi[2 * p + 1] = z1 * C.gisq[2 * p + 1];
  }
  __syncthreads();
  for (int j = threadIdx.x; j < beta; j += blockDim.x) {
    double w = 0.0;
    for (int64_t e = A.bptr[j]; e < A.bptr[j + 1]; ++e) w += scr[e];
    tv[j] = w - C.gam[j] * xi[j];
  }
  __syncthreads();
  if (want_v) {
    // scr[16 * j + q] = sum over k = q, q + 16, ... of S^{-1}_{jk} t_k
    for (int e = threadIdx.x; e < 16 * beta; e += blockDim.x) {
      const int j = e >> 4, q = e & 15;
      double a = 0.0;
#pragma unroll 8
      for (int k = q; k < beta; k += 16) a += A.SinvT[int64_t(k) * beta + j] * tv[k];
      scr[e] = a;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < beta; j += blockDim.x) {
      double a = 0.0;
      for (int q = 0; q < 16; ++q) a += scr[16 * j + q];
      vv[j] = xi[j] + a;
    }
  }
  const int ns = A.nsupp[dir];
  const double* __restrict__ GT = A.GT[dir];
  for (int r = threadIdx.x; r < ns; r += blockDim.x) {
    double acc = 0.0;
    int j = 0;
    for (; j + 16 <= beta; j += 16) {
      double g[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) g[u] = GT[int64_t(j + u) * ns + r];
#pragma unroll
      for (int u = 0; u < 16; ++u) acc += g[u] * tv[j + u];
    }
    for (; j < beta; ++j) acc += GT[int64_t(j) * ns + r] * tv[j];
    const int32_t at = A.supp[dir][r];
    th[at] = T(double(th[at]) - acc);
  }
  __syncthreads();
}

// f_{l-1} = P^T (f_l - A_l theta_l) - B_{l-1} v, residual staged in rbuf.
template <typename T>
__device__ void cv_restrict(const CoarseLevel& F, const CoarseLevel& Cl, const T* __restrict__ th,
                            const T* __restrict__ f, T* __restrict__ rbuf, T* __restrict__ fc,
                            const double* __restrict__ vv, int beta) {
  const Geom gf = F.g, gc = Cl.g;
  const T* __restrict__ coef = (const T*)F.coef;
  for (int lin = threadIdx.x; lin < gf.n * gf.n; lin += blockDim.x) {
    const int i1 = 1 + lin % gf.n, i2 = 1 + lin / gf.n;
    const int64_t ii = pidx(gf, i1, i2, 0);
    T r = f[ii];
#pragma unroll
    for (int t = 0; t < 9; ++t) r -= stencil_entry<T, 2>(coef, gf, t, ii) * th[ii + poff(gf, t % 3 - 1, t / 3 - 1, 0)];
    rbuf[ii] = r;
  }
  __syncthreads();
  LowRankRhs lr;
  if (beta) {
    lr.row_of = Cl.brow_of;
    lr.ptr = Cl.brptr;
    lr.col = Cl.brcol;
    lr.val = Cl.brval;
    lr.v = vv;
    lr.beta = beta;
  }
  for (int lin = threadIdx.x; lin < gc.n * gc.n; lin += blockDim.x) {
    const int J1 = 1 + lin % gc.n, J2 = 1 + lin / gc.n;
    const int64_t iJ = pidx(gc, J1, J2, 0);
    T acc = T(0);
#pragma unroll
    for (int t1 = 0; t1 < 9; ++t1) {
      const int ex = t1 % 3 - 1, ey = t1 / 3 - 1;
      acc += T(multilinear(ex, ey, 0)) * rbuf[pidx(gf, 2 * J1 + ex, 2 * J2 + ey, 0)];
    }
    fc[iJ] = T(double(acc) - lowrank_rhs(lr, 0, iJ));
  }
  __syncthreads();
}

// theta_l += P theta_{l-1} (multilinear), in the fixed four-term order of the
// fused post-sweep prolongation.
template <typename T>
__device__ void cv_prolong(const Geom& gf, const Geom& gc, T* __restrict__ th, const T* __restrict__ ps) {
  for (int lin = threadIdx.x; lin < gf.n * gf.n; lin += blockDim.x) {
    const int x = 1 + lin % gf.n, y = 1 + lin / gf.n;
    const int px = x & 1, py = y & 1;
    const int jx0 = x >> 1, jx1 = (x + 1) >> 1, jy0 = y >> 1, jy1 = (y + 1) >> 1;
    const T hx0 = px ? T(0.5) : T(1), hx1 = px ? T(0.5) : T(0);
    const T hy0 = py ? T(0.5) : T(1), hy1 = py ? T(0.5) : T(0);
    T s = (hx0 * hy0) * ps[pidx(gc, jx0, jy0, 0)];
    s += (hx1 * hy0) * ps[pidx(gc, jx1, jy0, 0)];
    s += (hx0 * hy1) * ps[pidx(gc, jx0, jy1, 0)];
    s += (hx1 * hy1) * ps[pidx(gc, jx1, jy1, 0)];
    const int64_t ii = pidx(gf, x, y, 0);
    th[ii] = th[ii] + s;
  }
  __syncthreads();
}

// theta_0 = K f_0 + U^{-1} z, 16 threads per row (loads unrolled by 8).
template <typename T>
__device__ void cv_coarsest(const CoarseLevel& A0, const CoarseCommon& C, T* __restrict__ th0,
                            const T* __restrict__ f0, double* __restrict__ fv,
                            double* __restrict__ zv, double* __restrict__ part, uint32_t m,
                            uint32_t chain) {
  const Geom g = A0.g;
  const int N0 = g.n * g.n;
  for (int k = threadIdx.x; k < N0; k += blockDim.x) {
    const int i1 = 1 + k % g.n, i2 = 1 + k / g.n;
    fv[k] = double(f0[pidx(g, i1, i2, 0)]);
  }
  for (int p = threadIdx.x; 2 * p < N0; p += blockDim.x) {
    const Block4 blk = philox10(uint32_t(p), 0u, m, 2u, C.seed, chain);
    double z0, z1;
    Gauss<double>::pair(blk, z0, z1);
    zv[2 * p] = z0;
    if (2 * p + 1 < N0) zv[2 * p + 1] = z1;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 16 * N0; e += blockDim.x) {
    const int r = e >> 4, q = e & 15;
    double s = 0.0;
#pragma unroll 8
    for (int k = q; k < N0; k += 16) {
      const double u = k >= r ? C.Uinv[int64_t(r) * N0 + k] : 0.0;
      s += C.K[int64_t(r) * N0 + k] * fv[k] + u * zv[k];
    }
    part[e] = s;
  }
  __syncthreads();
  for (int r = threadIdx.x; r < N0; r += blockDim.x) {
    double s = 0.0;
    for (int q = 0; q < 16; ++q) s += part[16 * r + q];
    th0[pidx(g, 1 + r % g.n, 1 + r / g.n, 0)] = T(s);
  }
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(kCT) void k_coarse_vcycle(CoarseArgs a) {
  extern __shared__ double smem[];
  const int c = blockIdx.x;
  const uint32_t m = uint32_t(*a.C.mcur);
  const uint32_t chain = a.C.chain0 + uint32_t(c);
  // LDS: per level theta and f (padded, T), residual scratch (T), then FP64
  // vectors for the low-rank and coarsest steps
  T* base = reinterpret_cast<T*>(smem);
  T* th[kMaxCoarseLevels];
  T* fl[kMaxCoarseLevels];
  int64_t off = 0;
  for (int l = 0; l <= a.lm; ++l) {
    th[l] = base + off;
    off += a.L[l].g.Np;
    fl[l] = base + off;
    off += a.L[l].g.Np;
  }
  T* rbuf = base + off;
  off += a.L[a.lm].g.Np;
  double* dbl = reinterpret_cast<double*>(base + ((off + 1) & ~int64_t(1)));
  double* xi = dbl;
  double* tv = xi + a.C.beta;
  double* vv = tv + a.C.beta;
  double* fv = vv + a.C.beta;
  double* zv = fv + a.L[0].g.n * a.L[0].g.n;
  double* part = zv + a.L[0].g.n * a.L[0].g.n;  // also the low-rank scratch
  for (int64_t e = threadIdx.x; e < off; e += blockDim.x) base[e] = T(0);
  __syncthreads();
  {  // right-hand side of level lm (restricted by the level above)
    const T* src = (const T*)a.f_top + int64_t(c) * a.L[a.lm].g.Np;
    for (int64_t e = threadIdx.x; e < a.L[a.lm].g.Np; e += blockDim.x) fl[a.lm][e] = src[e];
  }
  __syncthreads();
  for (int l = a.lm; l >= 1; --l) {
    for (int j = 0; j < a.C.nu1; ++j) {
      const uint32_t word = noise_word(l, j);
      cv_sweep<T>(a.L[l], th[l], fl[l], word, false, m, a.C.seed, chain);
      if (a.C.beta) cv_lowrank<T>(a.L[l], a.C, th[l], 0, word, j == a.C.nu1 - 1, xi, tv, vv, part, m, chain);
    }
    cv_restrict<T>(a.L[l], a.L[l - 1], th[l], fl[l], rbuf, fl[l - 1], vv, a.C.beta);
  }
  cv_coarsest<T>(a.L[0], a.C, th[0], fl[0], fv, zv, part, m, chain);
  for (int l = 1; l <= a.lm; ++l) {
    cv_prolong<T>(a.L[l].g, a.L[l - 1].g, th[l], th[l - 1]);
    for (int j = 0; j < a.C.nu2; ++j) {
      const uint32_t word = noise_word(l, a.C.nu1 + j);
      cv_sweep<T>(a.L[l], th[l], fl[l], word, true, m, a.C.seed, chain);
      if (a.C.beta) cv_lowrank<T>(a.L[l], a.C, th[l], 1, word, false, xi, tv, vv, part, m, chain);
    }
  }
  T* dst = (T*)a.theta_top + int64_t(c) * a.L[a.lm].g.Np;
  for (int64_t e = threadIdx.x; e < a.L[a.lm].g.Np; e += blockDim.x) dst[e] = th[a.lm][e];
}

}  // namespace

size_t coarse_vcycle_lds(const CoarseArgs& a, bool fp32, int64_t max_bnnz) {
  const size_t esz = fp32 ? 4 : 8;
  int64_t elems = 0;
  for (int l = 0; l <= a.lm; ++l) elems += 2 * a.L[l].g.Np;
  elems += a.L[a.lm].g.Np;
  elems += elems & 1;  // align the FP64 part
  const int64_t N0 = int64_t(a.L[0].g.n) * a.L[0].g.n;
  const int64_t part = std::max<int64_t>(std::max<int64_t>(16 * N0, 16 * int64_t(a.C.beta)), max_bnnz);
  return size_t(elems) * esz + size_t(3 * a.C.beta + 2 * N0 + part) * 8;
}

hipError_t coarse_vcycle_prepare(bool fp32, size_t lds_bytes) {
  if (fp32)
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_coarse_vcycle<float>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, int(lds_bytes));
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_coarse_vcycle<double>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, int(lds_bytes));
}

hipError_t launch_coarse_vcycle(const Launch& L, const CoarseArgs& a, size_t lds_bytes) {
  if (L.mcur == nullptr || L.dim != 2 || a.lm < 1 || a.lm >= kMaxCoarseLevels) return hipErrorInvalidValue;
  if (L.fp32)
    k_coarse_vcycle<float><<<L.nchains, kCT, lds_bytes, L.stream>>>(a);
  else
    k_coarse_vcycle<double><<<L.nchains, kCT, lds_bytes, L.stream>>>(a);
  return hipGetLastError();
}

}  // namespace mgmc
