// Learned prolongation: a small convolutional network on the coarse grid that
// maps the local coefficient to the weights of the finest transfer, with its
// training kernels (forward, backward, two-grid loss on crops, Adam).
//
// Any full-rank prolongation with Galerkin coarse operators leaves the
// sampler's target invariant (the invariance theorem of Sec. 4.2 holds for
// general P; Sec. 3.1 notes the transfers are not unique), so the network
// only changes the mixing speed.  The loss is the two-grid error reduction
// ||S_b T S_f e||_A^2 / ||e||_A^2 (T = I - P A_c^{-1} P^T A, A_c = P^T A P,
// S_f / S_b one noise-free red-black Gauss-Seidel sweep), averaged over crops
// and errors; k_crop_loss derives its gradient.
//
// Layout: features and activations [batch][channel][nc][nc] (FP32); network
// weights [cout][cin][9] + bias, the three layers concatenated; prolongation
// weights [nc*nc][9] (FP64), t = (dx+1) + 3 (dy+1), centre fixed to 1.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pnet.h"

namespace mgmc {
namespace {

constexpr int kB = 256;
constexpr int NIN = 24, NHID = 16, NOUT = 9;

__device__ __forceinline__ double softplus_d(double x) { return log1p(exp(-fabs(x))) + fmax(x, 0.0); }

// log a on the 24 faces around the fine 3x3 block of each coarse node
__global__ __launch_bounds__(kB) void k_features(const double* __restrict__ faces, int n,
                                                 float* __restrict__ X, int batch) {
  const int nc = (n - 1) / 2;
  const int64_t per = int64_t(n + 1) * n;
  const int64_t total = int64_t(batch) * nc * nc;
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= total) return;
  const int b = int(gid / (int64_t(nc) * nc));
  const int rem = int(gid % (int64_t(nc) * nc));
  const int Jx = 1 + rem % nc, Jy = 1 + rem / nc;
  const double* ax = faces + int64_t(b) * 2 * per;  // [y-1][face x], row length n+1
  const double* ay = ax + per;                        // [face y][x-1], row length n
  float* out = X + int64_t(b) * NIN * nc * nc + rem;
  const int64_t cs = int64_t(nc) * nc;
  int ch = 0;
  for (int r = 0; r < 3; ++r)
    for (int fi = 0; fi < 4; ++fi)
      out[(ch++) * cs] = float(log(ax[int64_t(2 * Jy - 2 + r) * (n + 1) + (2 * Jx - 2 + fi)]));
  for (int fr = 0; fr < 4; ++fr)
    for (int cx = 0; cx < 3; ++cx)
      out[(ch++) * cs] = float(log(ay[int64_t(2 * Jy - 2 + fr) * n + (2 * Jx - 2 + cx)]));
}

// out = conv3x3(in) + bias, zero padding; act = relu(out) if RELU
template <bool RELU>
__global__ __launch_bounds__(kB) void k_conv_fwd(const float* __restrict__ in, int cin,
                                                 const float* __restrict__ W,
                                                 const float* __restrict__ bias, int cout, int H,
                                                 int Wd, int batch, float* __restrict__ z,
                                                 float* __restrict__ act) {
  const int64_t hw = int64_t(H) * Wd;
  const int64_t total = int64_t(batch) * cout * hw;
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= total) return;
  const int x = int(gid % Wd), y = int((gid / Wd) % H);
  const int co = int((gid / hw) % cout), b = int(gid / (hw * cout));
  const float* ib = in + int64_t(b) * cin * hw;
  float acc = bias[co];
  for (int ci = 0; ci < cin; ++ci) {
    const float* wp = W + (int64_t(co) * cin + ci) * 9;
    const float* ip = ib + int64_t(ci) * hw;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int xx = x + t % 3 - 1, yy = y + t / 3 - 1;
      if (xx >= 0 && xx < Wd && yy >= 0 && yy < H) acc += wp[t] * ip[int64_t(yy) * Wd + xx];
    }
  }
  z[gid] = acc;
  if (RELU) act[gid] = acc > 0.f ? acc : 0.f;
}

// d in = conv3x3^T(d out), masked by relu'(z_in) when MASK
template <bool MASK>
__global__ __launch_bounds__(kB) void k_conv_bwd_data(const float* __restrict__ dout, int cout,
                                                      const float* __restrict__ W, int cin, int H,
                                                      int Wd, int batch,
                                                      const float* __restrict__ zin,
                                                      float* __restrict__ din) {
  const int64_t hw = int64_t(H) * Wd;
  const int64_t total = int64_t(batch) * cin * hw;
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= total) return;
  const int x = int(gid % Wd), y = int((gid / Wd) % H);
  const int ci = int((gid / hw) % cin), b = int(gid / (hw * cin));
  float acc = 0.f;
  for (int co = 0; co < cout; ++co) {
    const float* wp = W + (int64_t(co) * cin + ci) * 9;
    const float* dp = dout + (int64_t(b) * cout + co) * hw;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int xx = x - (t % 3 - 1), yy = y - (t / 3 - 1);
      if (xx >= 0 && xx < Wd && yy >= 0 && yy < H) acc += wp[t] * dp[int64_t(yy) * Wd + xx];
    }
  }
  if (MASK && !(zin[gid] > 0.f)) acc = 0.f;
  din[gid] = acc;
}

__device__ __forceinline__ double block_reduce(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (int(threadIdx.x) < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// dW[co][ci][t] = sum dout * shifted in; one block per weight (and per bias)
__global__ __launch_bounds__(kB) void k_conv_bwd_weight(const float* __restrict__ in, int cin,
                                                        const float* __restrict__ dout, int cout,
                                                        int H, int Wd, int batch,
                                                        float* __restrict__ dW,
                                                        float* __restrict__ db) {
  __shared__ double sh[kB];
  const int64_t hw = int64_t(H) * Wd;
  const int nw = cout * cin * 9;
  const int id = blockIdx.x;
  double acc = 0.0;
  if (id < nw) {
    const int t = id % 9, ci = (id / 9) % cin, co = id / (9 * cin);
    const int dx = t % 3 - 1, dy = t / 3 - 1;
    for (int64_t e = threadIdx.x; e < int64_t(batch) * hw; e += blockDim.x) {
      const int b = int(e / hw);
      const int p = int(e % hw);
      const int x = p % Wd, y = p / Wd;
      const int xx = x + dx, yy = y + dy;
      if (xx >= 0 && xx < Wd && yy >= 0 && yy < H)
        acc += double(dout[(int64_t(b) * cout + co) * hw + p]) *
               double(in[(int64_t(b) * cin + ci) * hw + int64_t(yy) * Wd + xx]);
    }
    const double s = block_reduce(acc, sh);
    if (threadIdx.x == 0) dW[id] = float(s);
  } else {
    const int co = id - nw;
    for (int64_t e = threadIdx.x; e < int64_t(batch) * hw; e += blockDim.x) {
      const int b = int(e / hw);
      acc += double(dout[(int64_t(b) * cout + co) * hw + e % hw]);
    }
    const double s = block_reduce(acc, sh);
    if (threadIdx.x == 0) db[co] = float(s);
  }
}

__device__ __forceinline__ double rho_at(const float* __restrict__ o, int nc, int Jx, int Jy, int t) {
  if (Jx < 1 || Jx > nc || Jy < 1 || Jy > nc) return 1.0;  // boundary ghost
  return softplus_d(double(o[int64_t(t) * nc * nc + int64_t(Jy - 1) * nc + (Jx - 1)]));
}

// covering coarse nodes of a fine coordinate: (J, d) with i = 2J + d
__device__ __forceinline__ int cover(int i, int* J, int* d) {
  if ((i & 1) == 0) {
    J[0] = i >> 1; d[0] = 0;
    return 1;
  }
  J[0] = (i - 1) >> 1; d[0] = 1;
  J[1] = (i + 1) >> 1; d[1] = -1;
  return 2;
}

__device__ __forceinline__ double z_at(const float* __restrict__ o, int nc, int ix, int iy) {
  int Jx[2], dx[2], Jy[2], dy[2];
  const int nx = cover(ix, Jx, dx), ny = cover(iy, Jy, dy);
  double z = 0.0;
  for (int a = 0; a < ny; ++a)
    for (int b = 0; b < nx; ++b) z += rho_at(o, nc, Jx[b], Jy[a], (dx[b] + 1) + 3 * (dy[a] + 1));
  return z;
}

// w[J][t] = rho_J(t) / Z(2J + delta_t), centre 1
__global__ __launch_bounds__(kB) void k_normalize(const float* __restrict__ O, int nc, int batch,
                                                  double* __restrict__ w) {
  const int64_t total = int64_t(batch) * nc * nc * 9;
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= total) return;
  const int t = int(gid % 9);
  const int64_t node = gid / 9;
  const int b = int(node / (int64_t(nc) * nc));
  const int rem = int(node % (int64_t(nc) * nc));
  const int Jx = 1 + rem % nc, Jy = 1 + rem / nc;
  const float* o = O + int64_t(b) * 9 * nc * nc;
  if (t == 4) {
    w[gid] = 1.0;
    return;
  }
  const int dx = t % 3 - 1, dy = t / 3 - 1;
  w[gid] = rho_at(o, nc, Jx, Jy, t) / z_at(o, nc, 2 * Jx + dx, 2 * Jy + dy);
}

// d o_J(t) = sigma(o_J(t)) (dw_J(t) - sum_{J' covering i} dw_J'(t') w_J'(t')) / Z(i)
__global__ __launch_bounds__(kB) void k_normalize_bwd(const float* __restrict__ O,
                                                      const double* __restrict__ w,
                                                      const double* __restrict__ dw, int nc,
                                                      int batch, float* __restrict__ dO) {
  const int64_t total = int64_t(batch) * nc * nc * 9;
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= total) return;
  const int t = int(gid % 9);
  const int64_t node = gid / 9;
  const int b = int(node / (int64_t(nc) * nc));
  const int rem = int(node % (int64_t(nc) * nc));
  const int Jx = 1 + rem % nc, Jy = 1 + rem / nc;
  const float* o = O + int64_t(b) * 9 * nc * nc;
  const double* wb = w + int64_t(b) * nc * nc * 9;
  const double* dwb = dw + int64_t(b) * nc * nc * 9;
  float* dob = dO + int64_t(b) * 9 * nc * nc;
  const int64_t oi = int64_t(t) * nc * nc + rem;
  if (t == 4) {
    dob[oi] = 0.f;
    return;
  }
  const int ix = 2 * Jx + (t % 3 - 1), iy = 2 * Jy + (t / 3 - 1);
  int Kx[2], ex[2], Ky[2], ey[2];
  const int nx = cover(ix, Kx, ex), ny = cover(iy, Ky, ey);
  double s = 0.0;
  for (int a = 0; a < ny; ++a)
    for (int c = 0; c < nx; ++c) {
      if (Kx[c] < 1 || Kx[c] > nc || Ky[a] < 1 || Ky[a] > nc) continue;
      const int64_t k = (int64_t(Ky[a] - 1) * nc + (Kx[c] - 1)) * 9 + (ex[c] + 1) + 3 * (ey[a] + 1);
      s += dwb[k] * wb[k];
    }
  const double x = double(o[oi]);
  const double sig = 1.0 / (1.0 + exp(-x));
  dob[oi] = float(sig * (dwb[node % (int64_t(nc) * nc) * 9 + t] - s) / z_at(o, nc, ix, iy));
}

// Two-grid loss on one crop of one field: coarse window of cw x cw nodes with
// origin J0, fine window [2 J0 - 1, 2 (J0 + cw - 1) + 1]^2, the fine operator
// restricted to the window (zero Dirichlet data outside).  For each error e:
//   e_s = S_f e, x = A_c^{-1} P^T A e_s, r = e_s - P x, u = S_b r,
//   loss += u^T A u / e^T A e,
//   W r = S_b^T A u = A u - A M_b^{-T} A u  (S_b = I - M_b^{-1} A),
//   y = A_c^{-1} P^T W r,
//   dL/dP += -2 [(W r - A P y) x^T + (A r) y^T] / e^T A e,
// with S_f / S_b one noise-free red-black Gauss-Seidel sweep (red = even
// coordinate sum first / last).  FP64 throughout; A_c is factored by a banded
// Cholesky (bandwidth cw + 1).
constexpr int kCW = 15, kFW = 2 * kCW + 1, kNF = kFW * kFW, kNCr = kCW * kCW, kBW = kCW + 1;

__global__ __launch_bounds__(kB) void k_crop_loss(const double* __restrict__ faces, int n,
                                                  double kappa2, const double* __restrict__ w,
                                                  const double* __restrict__ errors, int K,
                                                  int crops_x, double scale,
                                                  double* __restrict__ loss_out,
                                                  double* __restrict__ dw) {
  __shared__ double sA[5][kNF];   // fine stencil: centre, west, east, south, north
  __shared__ double sB[4][kNF];   // fine work vectors
  __shared__ double sL[kNCr][kBW + 1];  // band of the coarse matrix / its factor
  __shared__ double sG[kNCr], sX[kNCr], sY[kNCr], sYY[kNCr], sT[kNCr];
  __shared__ double scol[kBW + 1];
  __shared__ double sred[kB];
  const int b = blockIdx.y;
  const int crop = blockIdx.x;
  const int J0x = 1 + kCW * (crop % crops_x), J0y = 1 + kCW * (crop / crops_x);
  const int ix0 = 2 * J0x - 1, iy0 = 2 * J0y - 1;
  const int nc = (n - 1) / 2;
  const int64_t per = int64_t(n + 1) * n;
  const double* ax = faces + int64_t(b) * 2 * per;
  const double* ay = ax + per;
  const double* wb = w + int64_t(b) * nc * nc * 9;
  double* dwb = dw + int64_t(b) * nc * nc * 9;
  const double h = 1.0 / (n + 1), s = h * h, ih2 = 1.0 / (h * h);
  for (int r = threadIdx.x; r < kNF; r += blockDim.x) {
    const int x = ix0 + r % kFW, y = iy0 + r / kFW;
    const double aw = ax[int64_t(y - 1) * (n + 1) + (x - 1)], ae = ax[int64_t(y - 1) * (n + 1) + x];
    const double as = ay[int64_t(y - 1) * n + (x - 1)], an = ay[int64_t(y) * n + (x - 1)];
    const int lx = r % kFW, ly = r / kFW;
    sA[0][r] = s * (kappa2 + (aw + ae + as + an) * ih2);
    sA[1][r] = lx > 0 ? -s * aw * ih2 : 0.0;
    sA[2][r] = lx < kFW - 1 ? -s * ae * ih2 : 0.0;
    sA[3][r] = ly > 0 ? -s * as * ih2 : 0.0;
    sA[4][r] = ly < kFW - 1 ? -s * an * ih2 : 0.0;
  }
  for (int e = threadIdx.x; e < kNCr * (kBW + 1); e += blockDim.x) sL[e / (kBW + 1)][e % (kBW + 1)] = 0.0;
  __syncthreads();
  // P entry of crop coarse node (lx, ly) at offset t
  auto pw = [&](int lx, int ly, int t) { return wb[(int64_t(J0y + ly - 1) * nc + (J0x + lx - 1)) * 9 + t]; };
  // (A v)_r without the diagonal, and with it
  auto offdiag = [&](const double* v, int r) {
    const int lx = r % kFW, ly = r / kFW;
    double a = 0.0;
    if (lx > 0) a += sA[1][r] * v[r - 1];
    if (lx < kFW - 1) a += sA[2][r] * v[r + 1];
    if (ly > 0) a += sA[3][r] * v[r - kFW];
    if (ly < kFW - 1) a += sA[4][r] * v[r + kFW];
    return a;
  };
  auto Av = [&](const double* v, int r) { return sA[0][r] * v[r] + offdiag(v, r); };
  auto red = [&](int r) { return ((r % kFW + r / kFW) & 1) == 0; };  // window origin has an even sum
  // one colour of a noise-free Gauss-Seidel sweep for A u = 0, in place
  auto gs_colour = [&](double* u, bool want_red) {
    for (int r = threadIdx.x; r < kNF; r += blockDim.x)
      if (red(r) == want_red) u[r] = -offdiag(u, r) / sA[0][r];
    __syncthreads();
  };
  // (P^T v)_k for the crop's coarse nodes, into out
  auto restrict_to = [&](const double* v, double* out) {
    for (int k = threadIdx.x; k < kNCr; k += blockDim.x) {
      const int kx = k % kCW, ky = k / kCW;
      double g = 0.0;
      for (int t = 0; t < 9; ++t) g += pw(kx, ky, t) * v[(2 * kx + 1 + t % 3 - 1) + kFW * (2 * ky + 1 + t / 3 - 1)];
      out[k] = g;
    }
  };
  // (P c)_r at fine window site r
  auto prolong = [&](const double* c, int r) {
    const int fx = r % kFW, fy = r / kFW;
    double v = 0.0;
    for (int my = (fy - 2) / 2; my <= fy / 2; ++my)
      for (int mx = (fx - 2) / 2; mx <= fx / 2; ++mx) {
        if (mx < 0 || mx >= kCW || my < 0 || my >= kCW) continue;
        const int ddx = fx - (2 * mx + 1), ddy = fy - (2 * my + 1);
        if (ddx < -1 || ddx > 1 || ddy < -1 || ddy > 1) continue;
        v += pw(mx, my, (ddx + 1) + 3 * (ddy + 1)) * c[mx + kCW * my];
      }
    return v;
  };
  // A_c = P^T A P, 9-point: row of coarse node k, lower band entries
  for (int k = threadIdx.x; k < kNCr; k += blockDim.x) {
    const int kx = k % kCW, ky = k / kCW;
    double row[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int t1 = 0; t1 < 9; ++t1) {
      const int fx = 2 * kx + 1 + t1 % 3 - 1, fy = 2 * ky + 1 + t1 / 3 - 1;
      const double w1 = pw(kx, ky, t1);
      const int fi = fx + kFW * fy;
      const int nbx[5] = {fx, fx - 1, fx + 1, fx, fx};
      const int nby[5] = {fy, fy, fy, fy - 1, fy + 1};
      for (int q = 0; q < 5; ++q) {
        const double a = sA[q][fi];
        if (a == 0.0) continue;
        const int jx = nbx[q], jy = nby[q];
        // coarse nodes m of the crop covering fine (jx, jy): j = 2m + 1 + d (local)
        for (int my = ky - 1; my <= ky + 1; ++my)
          for (int mx = kx - 1; mx <= kx + 1; ++mx) {
            if (mx < 0 || mx >= kCW || my < 0 || my >= kCW) continue;
            const int ddx = jx - (2 * mx + 1), ddy = jy - (2 * my + 1);
            if (ddx < -1 || ddx > 1 || ddy < -1 || ddy > 1) continue;
            row[my - ky + 1][mx - kx + 1] += w1 * a * pw(mx, my, (ddx + 1) + 3 * (ddy + 1));
          }
      }
    }
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < 3; ++c) {
        const int mx = kx + c - 1, my = ky + a - 1;
        if (mx < 0 || mx >= kCW || my < 0 || my >= kCW) continue;
        const int m = mx + kCW * my;
        if (m <= k && k - m <= kBW) sL[k][k - m] = row[a][c];
      }
  }
  __syncthreads();
  // banded Cholesky A_c = L L^T in place (lower band), right-looking: column
  // k is scaled by 1 + kBW threads, then its rank-one update of the next kBW
  // rows is spread over the block
  for (int k = 0; k < kNCr; ++k) {
    const int tid = threadIdx.x;
    const double lkk = sqrt(sL[k][0]);
    if (tid <= kBW) scol[tid] = tid == 0 ? lkk : (k + tid < kNCr ? sL[k + tid][tid] / lkk : 0.0);
    __syncthreads();
    if (tid <= kBW && k + tid < kNCr) sL[k + tid][tid] = scol[tid];
    for (int p = tid; p < kBW * (kBW + 1) / 2; p += blockDim.x) {
      int a = 1;
      while (a * (a + 1) / 2 <= p) ++a;
      const int bb = p - a * (a - 1) / 2 + 1;  // 1 <= bb <= a <= kBW
      if (k + a < kNCr) sL[k + a][a - bb] -= scol[a] * scol[bb];
    }
    __syncthreads();
  }
  // out = A_c^{-1} g: column-oriented banded substitutions, one barrier per
  // unknown (out is the working right-hand side, tmp the forward result)
  auto solve = [&](const double* g, double* out, double* tmp) {
    for (int k = threadIdx.x; k < kNCr; k += blockDim.x) out[k] = g[k];
    __syncthreads();
    for (int k = 0; k < kNCr; ++k) {
      const int tid = threadIdx.x;
      const double yk = out[k] / sL[k][0];
      if (tid == 0) tmp[k] = yk;
      if (tid >= 1 && tid <= kBW && k + tid < kNCr) out[k + tid] -= sL[k + tid][tid] * yk;
      __syncthreads();
    }
    for (int k = kNCr - 1; k >= 0; --k) {
      const int tid = threadIdx.x;
      const double xk = tmp[k] / sL[k][0];
      if (tid == 0) out[k] = xk;
      if (tid >= 1 && tid <= kBW && k - tid >= 0) tmp[k - tid] -= sL[k][tid] * xk;
      __syncthreads();
    }
  };
  double* B0 = sB[0];
  double* B1 = sB[1];
  double* B2 = sB[2];
  double* B3 = sB[3];
  double crop_loss = 0.0;
  for (int q = 0; q < K; ++q) {
    const double* ef = errors + (int64_t(b) * K + q) * int64_t(n) * n;
    for (int r = threadIdx.x; r < kNF; r += blockDim.x) {
      const int x = ix0 + r % kFW, y = iy0 + r / kFW;
      B0[r] = ef[int64_t(y - 1) * n + (x - 1)];
    }
    __syncthreads();
    double part = 0.0;  // E = e^T A e
    for (int r = threadIdx.x; r < kNF; r += blockDim.x) part += B0[r] * Av(B0, r);
    const double E = block_reduce(part, sred);
    gs_colour(B0, true);   // e_s = S_f e
    gs_colour(B0, false);
    for (int r = threadIdx.x; r < kNF; r += blockDim.x) B1[r] = Av(B0, r);
    __syncthreads();
    restrict_to(B1, sG);   // g = P^T A e_s
    __syncthreads();
    solve(sG, sX, sY);     // x
    for (int r = threadIdx.x; r < kNF; r += blockDim.x) {
      const double rr = B0[r] - prolong(sX, r);  // r = e_s - P x
      B1[r] = rr;
      B2[r] = rr;
    }
    __syncthreads();
    gs_colour(B2, false);  // u = S_b r
    gs_colour(B2, true);
    part = 0.0;
    for (int r = threadIdx.x; r < kNF; r += blockDim.x) {
      const double v = Av(B2, r);
      B3[r] = v;           // v = A u
      part += B2[r] * v;
    }
    const double uAu = block_reduce(part, sred);
    crop_loss += uAu / E;
    // z = M_b^{-T} v: red sites first (no coupling), then black from red
    for (int r = threadIdx.x; r < kNF; r += blockDim.x)
      if (red(r)) B0[r] = B3[r] / sA[0][r];
    __syncthreads();
    for (int r = threadIdx.x; r < kNF; r += blockDim.x)
      if (!red(r)) B0[r] = (B3[r] - offdiag(B0, r)) / sA[0][r];
    __syncthreads();
    for (int r = threadIdx.x; r < kNF; r += blockDim.x) B2[r] = B3[r] - Av(B0, r);  // W r
    __syncthreads();
    restrict_to(B2, sT);   // P^T W r
    __syncthreads();
    solve(sT, sYY, sY);    // y
    for (int r = threadIdx.x; r < kNF; r += blockDim.x) B3[r] = prolong(sYY, r);  // P y
    __syncthreads();
    for (int r = threadIdx.x; r < kNF; r += blockDim.x) B0[r] = B2[r] - Av(B3, r);  // W r - A P y
    __syncthreads();
    for (int r = threadIdx.x; r < kNF; r += blockDim.x) B3[r] = Av(B1, r);  // A r
    __syncthreads();
    for (int k = threadIdx.x; k < kNCr; k += blockDim.x) {
      const int kx = k % kCW, ky = k / kCW;
      const int64_t base = (int64_t(J0y + ky - 1) * nc + (J0x + kx - 1)) * 9;
      for (int t = 0; t < 9; ++t) {
        const int i = (2 * kx + 1 + t % 3 - 1) + kFW * (2 * ky + 1 + t / 3 - 1);
        dwb[base + t] += -2.0 * scale * (B0[i] * sX[k] + B3[i] * sYY[k]) / E;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) loss_out[int64_t(b) * gridDim.x + crop] = crop_loss * scale;
}

// deterministic sum of the per-crop losses (one block)
__global__ __launch_bounds__(kB) void k_sum(const double* __restrict__ x, int64_t n,
                                            double* __restrict__ out) {
  __shared__ double sh[kB];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) acc += x[i];
  const double s = block_reduce(acc, sh);
  if (threadIdx.x == 0) out[0] = s;
}

__global__ void k_fill_d(double* p, int64_t n, double v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ __launch_bounds__(kB) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                             float* __restrict__ m, float* __restrict__ v, int np,
                                             float lr, float b1, float b2, float eps, float c1,
                                             float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

inline unsigned nblk(int64_t n) { return unsigned((n + kB - 1) / kB); }

}  // namespace

int64_t pnet_param_count() {
  return int64_t(NHID) * NIN * 9 + NHID + int64_t(NHID) * NHID * 9 + NHID + int64_t(NOUT) * NHID * 9 + NOUT;
}

hipError_t pnet_forward(const PnetBuffers& P, const double* faces, int batch, hipStream_t st) {
  const int nc = (P.n - 1) / 2;
  const int64_t hw = int64_t(nc) * nc;
  const float* W1 = P.params;
  const float* b1 = W1 + NHID * NIN * 9;
  const float* W2 = b1 + NHID;
  const float* b2 = W2 + NHID * NHID * 9;
  const float* W3 = b2 + NHID;
  const float* b3 = W3 + NOUT * NHID * 9;
  k_features<<<nblk(batch * hw), kB, 0, st>>>(faces, P.n, P.x0, batch);
  k_conv_fwd<true><<<nblk(batch * NHID * hw), kB, 0, st>>>(P.x0, NIN, W1, b1, NHID, nc, nc, batch, P.z1, P.a1);
  k_conv_fwd<true><<<nblk(batch * NHID * hw), kB, 0, st>>>(P.a1, NHID, W2, b2, NHID, nc, nc, batch, P.z2, P.a2);
  k_conv_fwd<false><<<nblk(batch * NOUT * hw), kB, 0, st>>>(P.a2, NHID, W3, b3, NOUT, nc, nc, batch, P.o, nullptr);
  k_normalize<<<nblk(batch * hw * 9), kB, 0, st>>>(P.o, nc, batch, P.w);
  return hipGetLastError();
}

hipError_t pnet_loss_grad(const PnetBuffers& P, const double* faces, const double* errors,
                          int batch, int K, double kappa2, hipStream_t st) {
  const int nc = (P.n - 1) / 2;
  const int64_t hw = int64_t(nc) * nc;
  const int cx = nc / kCW;
  if (cx < 1) return hipErrorInvalidValue;
  hipError_t e = pnet_forward(P, faces, batch, st);
  if (e != hipSuccess) return e;
  k_fill_d<<<nblk(batch * hw * 9), kB, 0, st>>>(P.dw, batch * hw * 9, 0.0);
  const double scale = 1.0 / (double(batch) * cx * cx * K);
  dim3 grid(unsigned(cx * cx), unsigned(batch));
  k_crop_loss<<<grid, kB, 0, st>>>(faces, P.n, kappa2, P.w, errors, K, cx, scale, P.loss, P.dw);
  k_sum<<<1, kB, 0, st>>>(P.loss, int64_t(batch) * cx * cx, P.loss_total);
  k_normalize_bwd<<<nblk(batch * hw * 9), kB, 0, st>>>(P.o, P.w, P.dw, nc, batch, P.do_);
  float* g = P.grad;
  float* gW1 = g;
  float* gb1 = gW1 + NHID * NIN * 9;
  float* gW2 = gb1 + NHID;
  float* gb2 = gW2 + NHID * NHID * 9;
  float* gW3 = gb2 + NHID;
  float* gb3 = gW3 + NOUT * NHID * 9;
  const float* W2 = P.params + NHID * NIN * 9 + NHID;
  const float* W3 = W2 + NHID * NHID * 9 + NHID;
  k_conv_bwd_weight<<<NOUT * NHID * 9 + NOUT, kB, 0, st>>>(P.a2, NHID, P.do_, NOUT, nc, nc, batch, gW3, gb3);
  k_conv_bwd_data<true><<<nblk(batch * NHID * hw), kB, 0, st>>>(P.do_, NOUT, W3, NHID, nc, nc, batch, P.z2, P.d2);
  k_conv_bwd_weight<<<NHID * NHID * 9 + NHID, kB, 0, st>>>(P.a1, NHID, P.d2, NHID, nc, nc, batch, gW2, gb2);
  k_conv_bwd_data<true><<<nblk(batch * NHID * hw), kB, 0, st>>>(P.d2, NHID, W2, NHID, nc, nc, batch, P.z1, P.d1);
  k_conv_bwd_weight<<<NHID * NIN * 9 + NHID, kB, 0, st>>>(P.x0, NIN, P.d1, NHID, nc, nc, batch, gW1, gb1);
  return hipGetLastError();
}

hipError_t pnet_adam(const PnetBuffers& P, float lr, int step, hipStream_t st) {
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, float(step)), c2 = 1.f - powf(b2, float(step));
  const int np = int(pnet_param_count());
  k_adam<<<nblk(np), kB, 0, st>>>(P.params, P.grad, P.m, P.v, np, lr, b1, b2, 1e-8f, c1, c2);
  return hipGetLastError();
}

int pnet_crops_per_field(int n) {
  const int nc = (n - 1) / 2;
  return (nc / kCW) * (nc / kCW);
}

}  // namespace mgmc
