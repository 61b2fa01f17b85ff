// Counter-based Gaussian noise on the device: Philox4x32-10 (Salmon, Moraes,
// Dror, Shaw, SC'11) and the Box-Muller transform.
//
// One Philox block gives two normals: u1 from words (x0, x1), u2 from (x2, x3)
// as the top 53 bits plus half an ulp scaled by 2^-53; z = sqrt(-2 ln u1)
// (cos, sin)(2 pi u2).  The double-precision logarithm and sine/cosine are
// short series written out here (few live registers inside the sweeps).  The
// single-precision variant forms the same uniforms (see Gauss<float>), so its
// normals track the double ones to float rounding from the same counters.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mgmc {

struct Block4 {
  uint32_t x0, x1, x2, x3;
};

__device__ __forceinline__ Block4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                           uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // one 32 x 32 -> 64-bit multiply gives both halves of each product
    const uint64_t pa = uint64_t(0xD2511F53u) * c0;
    const uint64_t pb = uint64_t(0xCD9E8D57u) * c2;
    const uint32_t n0 = uint32_t(pb >> 32) ^ c1 ^ k0;
    const uint32_t n2 = uint32_t(pa >> 32) ^ c3 ^ k1;
    c0 = n0;
    c1 = uint32_t(pb);
    c2 = n2;
    c3 = uint32_t(pa);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return Block4{c0, c1, c2, c3};
}

template <typename T>
struct Gauss;

// Natural logarithm of u in (0, 1), a normal double.  u = f 2^k with f in
// [1/sqrt 2, sqrt 2); with s = (f - 1) / (f + 1), log f = 2 atanh s =
// 2 s sum_j s^(2j) / (2j + 1), and |s| <= 0.1716 makes ten terms accurate to
// 3e-17 relative.  Horner form keeps few values live.
__device__ __forceinline__ double log_unit(double u) {
  int k;
  double f = frexp(u, &k);  // f in [0.5, 1)
  if (f < 0.70710678118654752440) {
    f *= 2.0;
    k -= 1;
  }
  const double s = (f - 1.0) / (f + 1.0);
  const double s2 = s * s;
  double p = 1.0 / 19.0;
  p = fma(p, s2, 1.0 / 17.0);
  p = fma(p, s2, 1.0 / 15.0);
  p = fma(p, s2, 1.0 / 13.0);
  p = fma(p, s2, 1.0 / 11.0);
  p = fma(p, s2, 1.0 / 9.0);
  p = fma(p, s2, 1.0 / 7.0);
  p = fma(p, s2, 1.0 / 5.0);
  p = fma(p, s2, 1.0 / 3.0);
  p = fma(p, s2, 1.0);
  return fma(double(k), 0.69314718055994530942, 2.0 * s * p);
}

// Square root of a positive double that is neither tiny (below 2^-767) nor
// infinite: the hardware reciprocal square root refined by the Newton steps
// of the general sequence, without its rescaling of tiny arguments and its
// checks for zero and infinity (the Box-Muller radicand -2 ln u lies in
// [2^-53, 75]), so the result is the same as sqrt() for such arguments.
__device__ __forceinline__ double sqrt_normal(double a) {
  const double y = __builtin_amdgcn_rsq(a);
  double s = a * y;
  double h = 0.5 * y;
  const double r = fma(-h, s, 0.5);
  s = fma(s, r, s);
  h = fma(h, r, h);
  double d = fma(-s, s, a);
  s = fma(d, h, s);
  d = fma(-s, s, a);
  return fma(d, h, s);
}

// sin and cos of 2 pi u for u in [0, 1).  t = 4u is exact; with q the
// nearest integer and r = t - q (exact, |r| <= 1/2) the angle is
// q pi/2 + x, x = r pi/2 in [-pi/4, pi/4], where Taylor series of nine
// (sin) and ten (cos) terms are accurate to 1e-19 and 3e-21.
__device__ __forceinline__ void sincos_2pi(double u, double& sn, double& cs) {
  const double t = 4.0 * u;
  const double qd = rint(t);
  const double x = (t - qd) * 1.57079632679489661923;
  const double x2 = x * x;
  double ps = 1.0 / 355687428096000.0;  // 1/17!
  ps = fma(ps, x2, -1.0 / 1307674368000.0);
  ps = fma(ps, x2, 1.0 / 6227020800.0);
  ps = fma(ps, x2, -1.0 / 39916800.0);
  ps = fma(ps, x2, 1.0 / 362880.0);
  ps = fma(ps, x2, -1.0 / 5040.0);
  ps = fma(ps, x2, 1.0 / 120.0);
  ps = fma(ps, x2, -1.0 / 6.0);
  ps = fma(ps, x2, 1.0);
  const double sx = x * ps;
  double pc = 1.0 / 6402373705728000.0;  // 1/18!
  pc = fma(pc, x2, -1.0 / 20922789888000.0);
  pc = fma(pc, x2, 1.0 / 87178291200.0);
  pc = fma(pc, x2, -1.0 / 479001600.0);
  pc = fma(pc, x2, 1.0 / 3628800.0);
  pc = fma(pc, x2, -1.0 / 40320.0);
  pc = fma(pc, x2, 1.0 / 720.0);
  pc = fma(pc, x2, -1.0 / 24.0);
  pc = fma(pc, x2, 0.5);
  const double cx = fma(-x2, pc, 1.0);
  const int q = int(qd) & 3;
  const double a = (q & 1) ? cx : sx;  // sin of the angle up to sign
  const double b = (q & 1) ? sx : cx;  // cos of the angle up to sign
  sn = (q & 2) ? -a : a;
  cs = (q == 1 || q == 2) ? -b : b;
}

// Table-driven double-precision Box-Muller for kernels that stage the table
// in LDS.  Layout (kBmTable = 770 doubles, filled by fill_bm_table on the
// host):
//   [0, 128)     log c_i,  c_i = 45/64 + (i + 1/2) 45/8192, the midpoints of
//                128 equal cells covering [45/64, 45/32)
//   [128, 256)   1 / c_i
//   [256, 513)   sin(2 pi k / 256), k = 0..256
//   [513, 770)   cos(2 pi k / 256)
// log u: u = f 2^e with f in [45/64, 45/32); with c the midpoint of f's cell,
// r = (f - c) / c has |r| <= 1/256 and log u = e ln 2 + log c + log1p r,
// log1p r to seven terms (error < r^8 / 8).  sin/cos(2 pi u): t = 256 u
// (exact), k = nearest integer, x = (t - k) 2 pi / 256 with |x| <= pi/256,
// short series for sin x and cos x, and the angle-sum formulas with the
// tabulated sin and cos of 2 pi k / 256.
__device__ __forceinline__ void gauss_pair_tab(const Block4& x, const double* __restrict__ tab,
                                               double& z0, double& z1) {
  const uint64_t w1 = (uint64_t(x.x0) << 32) | uint64_t(x.x1);
  const uint64_t w2 = (uint64_t(x.x2) << 32) | uint64_t(x.x3);
  const double u1 = (double(w1 >> 11) + 0.5) * 0x1p-53;
  const double u2 = (double(w2 >> 11) + 0.5) * 0x1p-53;
  int e;
  double f = frexp(u1, &e);  // [0.5, 1)
  if (f < 0.703125) {
    f *= 2.0;
    e -= 1;
  }
  const int i = min(int((f - 0.703125) * (8192.0 / 45.0)), 127);
  const double c = 0.703125 + (double(i) + 0.5) * (45.0 / 8192.0);
  const double r = (f - c) * tab[128 + i];
  double p = 1.0 / 7.0;
  p = fma(p, r, -1.0 / 6.0);
  p = fma(p, r, 1.0 / 5.0);
  p = fma(p, r, -0.25);
  p = fma(p, r, 1.0 / 3.0);
  p = fma(p, r, -0.5);
  p = fma(p, r, 1.0);
  const double lg = fma(double(e), 0.69314718055994530942, fma(r, p, tab[i]));
  const double rad = sqrt_normal(-2.0 * lg);
  const double t = u2 * 256.0;
  const double kd = rint(t);
  const int k = int(kd);
  const double xa = (t - kd) * 0.024543692606170259675;  // 2 pi / 256
  const double x2 = xa * xa;
  double ps = -1.0 / 5040.0;
  ps = fma(ps, x2, 1.0 / 120.0);
  ps = fma(ps, x2, -1.0 / 6.0);
  const double sx = fma(xa * x2, ps, xa);
  double pc = -1.0 / 720.0;
  pc = fma(pc, x2, 1.0 / 24.0);
  pc = fma(pc, x2, -0.5);
  const double cx = fma(x2, pc, 1.0);
  const double sk = tab[256 + k], ck = tab[513 + k];
  const double sn = fma(sk, cx, ck * sx);
  const double cs = fma(ck, cx, -(sk * sx));
  z0 = rad * cs;
  z1 = rad * sn;
}

template <>
struct Gauss<double> {
  static __device__ __forceinline__ void pair(const Block4& x, double& z0, double& z1) {
    const uint64_t w1 = (uint64_t(x.x0) << 32) | uint64_t(x.x1);
    const uint64_t w2 = (uint64_t(x.x2) << 32) | uint64_t(x.x3);
    const double u1 = (double(w1 >> 11) + 0.5) * 0x1p-53;
    const double u2 = (double(w2 >> 11) + 0.5) * 0x1p-53;
    const double rad = sqrt_normal(-2.0 * log_unit(u1));
    double sn, cs;
    sincos_2pi(u2, sn, cs);
    z0 = rad * cs;
    z1 = rad * sn;
  }
};

// sin and cos of 2 pi u in single precision for u in [0, 1): t = 4u is exact;
// with q the nearest integer and r = t - q (exact, |r| <= 1/2) the angle is
// q pi/2 + x, x = r pi/2 in [-pi/4, pi/4], where the Taylor series to x^9
// (sin) and x^10 (cos) leave truncation errors below 2e-9 and 2e-10.
__device__ __forceinline__ void sincos_2pi_f(float u, float& sn, float& cs) {
  const float t = 4.0f * u;
  const float qf = rintf(t);
  const float x = (t - qf) * 1.57079632679489661923f;
  const float x2 = x * x;
  float ps = 1.0f / 362880.0f;  // 1/9!
  ps = fmaf(ps, x2, -1.0f / 5040.0f);
  ps = fmaf(ps, x2, 1.0f / 120.0f);
  ps = fmaf(ps, x2, -1.0f / 6.0f);
  const float sx = fmaf(x * x2, ps, x);
  float pc = -1.0f / 3628800.0f;  // -1/10!
  pc = fmaf(pc, x2, 1.0f / 40320.0f);
  pc = fmaf(pc, x2, -1.0f / 720.0f);
  pc = fmaf(pc, x2, 1.0f / 24.0f);
  pc = fmaf(pc, x2, -0.5f);
  const float cx = fmaf(x2, pc, 1.0f);
  const int q = int(qf) & 3;
  const float a = (q & 1) ? cx : sx;  // sin of the angle up to sign
  const float b = (q & 1) ? sx : cx;  // cos of the angle up to sign
  sn = (q & 2) ? -a : a;
  cs = (q == 1 || q == 2) ? -b : b;
}

// Single precision from the same 53-bit uniforms as the double path, so that
// the two differ by float rounding only.  u = hi + lo with hi = (x0 >> 8)
// 2^-24 (exact in float) and 0 < lo < 2^-24 the remaining 29 bits plus half
// an ulp; ln u = ln hi + lo / hi (the dropped terms of log1p are below
// 2^-25 absolute, since lo / hi <= 2^-12) when hi >= 2^-12, else ln(hi + lo)
// directly (|ln u| > 8 there).  The angle 2 pi u2 = 2 pi hi2 + 2 pi lo2 is
// applied as sin/cos of the first part rotated by the small second one.
// Radius and angle thus carry float rounding relative to the double
// transform, not the 24-bit truncation of u.
//
// The logarithm, reciprocal and square root are the hardware instructions
// (v_log_f32 as log2 times ln 2, v_rcp_f32, v_sqrt_f32, each within about
// one ulp) rather than the library's correctly rounded sequences: their
// arguments here are never denormal or zero (u >= 2^-54, -2 ln u >= 2^-24),
// which is all those sequences add, and the noise kernels are bound by
// vector instruction issue.  For the same reason sin and cos come from the
// short series above instead of the library's general argument reduction.
template <>
struct Gauss<float> {
  static __device__ __forceinline__ void pair(const Block4& x, float& z0, float& z1) {
    const float h1 = float(x.x0 >> 8) * 0x1p-24f;
    const float l1 = (float(((x.x0 & 0xffu) << 21) | (x.x1 >> 11)) + 0.5f) * 0x1p-53f;
    const bool big = h1 >= 0x1p-12f;
    const float lg = __builtin_amdgcn_logf(big ? h1 : h1 + l1) * 0.693147180559945309f +
                     (big ? l1 * __builtin_amdgcn_rcpf(h1) : 0.0f);
    const float rad = __builtin_amdgcn_sqrtf(-2.0f * lg);
    const float h2 = float(x.x2 >> 8) * 0x1p-24f;
    const float l2 = (float(((x.x2 & 0xffu) << 21) | (x.x3 >> 11)) + 0.5f) * 0x1p-53f;
    float sn, cs;
    sincos_2pi_f(h2, sn, cs);
    const float d = 6.28318530717958647692f * l2;
    z0 = rad * fmaf(-d, sn, cs);
    z1 = rad * fmaf(d, cs, sn);
  }
};

}  // namespace mgmc
