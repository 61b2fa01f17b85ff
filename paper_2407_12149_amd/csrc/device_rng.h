// Counter-based Gaussian noise on the device: Philox4x32-10 (Salmon, Moraes,
// Dror, Shaw, SC'11) and the Box-Muller transform.
//
// One Philox block gives two normals: u1 from words (x0, x1), u2 from (x2, x3)
// as the top 53 bits plus half an ulp scaled by 2^-53; z = sqrt(-2 ln u1)
// (cos, sin)(2 pi u2).  The single-precision variant takes the top 24 bits of
// x0 and x2, so its normals track the double ones to ~1e-7 from the same
// counters.
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

template <>
struct Gauss<double> {
  static __device__ __forceinline__ void pair(const Block4& x, double& z0, double& z1) {
    const uint64_t w1 = (uint64_t(x.x0) << 32) | uint64_t(x.x1);
    const uint64_t w2 = (uint64_t(x.x2) << 32) | uint64_t(x.x3);
    const double u1 = (double(w1 >> 11) + 0.5) * 0x1p-53;
    const double u2 = (double(w2 >> 11) + 0.5) * 0x1p-53;
    const double rad = sqrt(-2.0 * log(u1));
    // (sin, cos)(2 pi u2) via the pi-scaled forms: exact argument reduction
    double sn, cs;
    sincospi(2.0 * u2, &sn, &cs);
    z0 = rad * cs;
    z1 = rad * sn;
  }
};

template <>
struct Gauss<float> {
  static __device__ __forceinline__ void pair(const Block4& x, float& z0, float& z1) {
    const float u1 = (float(x.x0 >> 8) + 0.5f) * 0x1p-24f;
    const float u2 = (float(x.x2 >> 8) + 0.5f) * 0x1p-24f;
    const float rad = sqrtf(-2.0f * logf(u1));
    float sn, cs;
    sincospif(2.0f * u2, &sn, &cs);
    z0 = rad * cs;
    z1 = rad * sn;
  }
};

}  // namespace mgmc
