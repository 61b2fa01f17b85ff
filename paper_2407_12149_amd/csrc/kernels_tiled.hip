// LDS-tiled 2D kernels: one launch per smoother sweep and per restriction.
//
// k_sweep2d_tiled runs every colour pass of one random Gauss-Seidel sweep
// (Alg. 2/3 with M = D + L in colour order) on a TX x TY tile held in LDS
// with a halo of NPASS sites: pass p updates the tile plus a ring of
// NPASS-1-p sites, so after the last pass the tile interior is exactly what
// NPASS global passes would give (neighbouring tiles recompute the shared
// ring identically: the noise is counter-based).  NPASS = 2 is red-black on
// the 5-point finest stencil (colours of equal parity sum never couple), 4 is
// the four-colour order on 9-point Galerkin stencils.  Each block loops over
// a group of chains, so the operator is read from HBM once per sweep and hit
// in cache for the remaining chains.  With PROLONG the coarse-grid correction
// theta += P psi (Alg. 1, prolongation step) is applied while the tile is
// loaded, fusing it into the post-smoother.
//
// k_restrict2d_reg computes f_{l-1} = P^T (f_l - A_l theta) (Alg. 1,
// restriction step) for a tile of coarse nodes from fine residuals staged
// in LDS, with the residual's operator held in registers across chains.
#include <cmath>

#include "device_common.h"
#include "device_rng.h"
#include "mgmc_internal.h"

namespace mgmc {

namespace {

constexpr int kFwdOrder2[4] = {0, 3, 1, 2};

// (P psi)(x, y) for fine node (x, y): the coarse nodes J with |x - 2 J| <= 1
// per axis are J0 = x >> 1 (offset x & 1) and, for odd x, J1 = (x + 1) >> 1
// (offset -1); for even x, J1 = J0, so every node takes the same four reads.
// User weights: J1 = J0 enters with weight 0 and the sum runs in a fixed
// order (J0y,J0x), (J0y,J1x), (J1y,J0x), (J1y,J1x).  get(jx, jy) reads psi
// at coarse node (jx, jy).
template <typename T, bool USERP, class Get>
__device__ __forceinline__ T prolong_sum(Get get, const Geom& gc, const double* __restrict__ wP,
                                         int x, int y) {
  const int px = x & 1, py = y & 1;
  const int jx0 = x >> 1, jx1 = (x + 1) >> 1, jy0 = y >> 1, jy1 = (y + 1) >> 1;
  const T v00 = get(jx0, jy0), v01 = get(jx1, jy0), v10 = get(jx0, jy1), v11 = get(jx1, jy1);
  if (!USERP) {
    // bilinear (weights 1, 1/2, 1/4): with J1 = J0 on an even axis, a
    // quarter of the four reads is the interpolant in every parity case; it
    // rounds like the weighted sum unless x and y are both odd
    return T(0.25) * ((v00 + v10) + (v01 + v11));
  }
  auto W = [&](int jx, int jy, int dx, int dy) {
    return T(wP[int64_t((dx + 1) + 3 * (dy + 1)) * gc.Np + pidx(gc, jx, jy, 0)]);
  };
  const T w00 = W(jx0, jy0, px, py);
  const T w01 = px ? W(jx1, jy0, -1, py) : T(0);
  const T w10 = py ? W(jx0, jy1, px, -1) : T(0);
  const T w11 = (px && py) ? W(jx1, jy1, -1, -1) : T(0);
  T s = w00 * v00;
  s += w01 * v01;
  s += w10 * v10;
  s += w11 * v11;
  return s;
}

template <typename T, bool USERP>
__device__ __forceinline__ T prolong_at(const T* __restrict__ ps, const Geom& gc,
                                        const double* __restrict__ wP, int x, int y) {
  return prolong_sum<T, USERP>([&](int jx, int jy) { return ps[pidx(gc, jx, jy, 0)]; }, gc, wP, x, y);
}

// The same from a coarse patch staged in LDS: sp holds the coarse nodes J
// with J - (jx0, jy0) in [0, cw) x [0, ch), row-major.
template <typename T, bool USERP>
__device__ __forceinline__ T prolong_lds(const T* __restrict__ sp, int cw, int jx0, int jy0,
                                         const Geom& gc, const double* __restrict__ wP, int x,
                                         int y) {
  return prolong_sum<T, USERP>([&](int jx, int jy) { return sp[(jy - jy0) * cw + (jx - jx0)]; }, gc,
                               wP, x, y);
}

// Workgroup barrier for LDS traffic only: waits for this wave's LDS
// operations, not for outstanding vector-memory operations, so LDS DMA
// copies into another buffer stay in flight across it.  (A fenced
// __syncthreads would wait for them, the DMA writing LDS.)  The memory
// clobber keeps the compiler from moving memory accesses across it.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// 16 bytes per lane from memory into LDS (lane l of the wavefront fills
// bytes 16 l .. 16 l + 15 after dst, dst the same in every lane); the copy
// completes asynchronously, tracked by the vector-memory counter.
__device__ __forceinline__ void lds_dma16(const void* src, void* dst) {
#if defined(__HIP_DEVICE_COMPILE__)
  __builtin_amdgcn_global_load_lds(src, dst, 16, 0, 0);
#endif
}

// LDS layout of a tile row: four sub-rows by x mod 4, each of odd length W,
// so the lanes of a wavefront (pairs four sites apart, the same x mod 4)
// read consecutive words and neighbour reads are free of bank conflicts.
// The row stride RS is padded to 9 mod 16 elements (ESZ = 8) or mod 32
// (ESZ = 4): a segment-sweep wavefront holds 18 segments of each of rows
// two apart, and 2 RS = 18 (mod 32 bank pairs / 64 banks) puts lane u on
// bank (pair) u mod 32 (mod 64) whichever rows the lanes fall in.
template <int RX, int ESZ>
struct Swz {
  static constexpr int W = ((RX + 3) / 4) | 1;
  static constexpr int MB = ESZ == 8 ? 16 : 32;
  static constexpr int RS = 4 * W + ((9 - 4 * W) % MB + MB) % MB;  // row stride
  static __device__ __forceinline__ int pos(int lx, int ly) { return ly * RS + (lx & 3) * W + (lx >> 2); }
  // offsets of the x-neighbours of a site with lx & 3 == s
  static __device__ __forceinline__ int east(int s) { return s < 3 ? W : 1 - 3 * W; }
  static __device__ __forceinline__ int west(int s) { return s > 0 ? -W : 3 * W - 1; }
};

// Write B's weight times the swept value of chain c at B's sites inside
// tile `tile` into the snapshot (B^T theta is then formed from it without
// another pass over theta).  at(lx, ly) reads the LDS tile at region
// coordinates.
template <class At>
__device__ __forceinline__ void snap_sites(const BSnap& bs, const Geom& g, int tile, int c, int ox,
                                           int oy, int nt, At at) {
  const int b0 = bs.ptr[tile], b1 = bs.ptr[tile + 1];
  for (int i = b0 + int(threadIdx.x); i < b1; i += nt) {
    const int e = bs.ent[i];
    const int site = bs.idx[e];
    const int x = site % g.px - 3, y = site / g.px;
    bs.snap[int64_t(c) * bs.nnz + e] = bs.w[e] * at(x - ox, y - oy);
  }
}

template <typename T, int NPASS, bool PROLONG, bool USERP, int TX, int TY>
__global__ __launch_bounds__(kBlock) void k_sweep2d_tiled(
    const T* __restrict__ coef, const T* __restrict__ invd, const T* __restrict__ isqd,
    const T* __restrict__ theta_in, T* __restrict__ theta_out, int zero_in,
    const T* __restrict__ f, int64_t fcs, Geom g,
    const T* __restrict__ psi, Geom gc, const double* __restrict__ wP, int backward,
    uint32_t word, const int64_t* __restrict__ mcur, uint32_t seed, uint32_t chain0, int tiles_x,
    int cpb, int nchains, BSnap bs) {
  constexpr bool CROSS = (NPASS == 2);
  constexpr int H = NPASS, RX = TX + 2 * H, RY = TY + 2 * H;
  constexpr int Q = RX / 4 + 2;  // pair slots per row
  using Z = Swz<RX, int(sizeof(T))>;
  __shared__ T sh[RY * Z::RS];
  const int n = g.n;
  const int tx0 = int(blockIdx.x % tiles_x) * TX + 1;
  const int ty0 = int(blockIdx.x / tiles_x) * TY + 1;
  const int ox = tx0 - H, oy = ty0 - H;
  const uint32_t m = uint32_t(*mcur);
  const int cb = int(blockIdx.y) * cpb;
  const int ce = min(nchains, cb + cpb);
  for (int c = cb; c < ce; ++c) {
    const T* thi = theta_in + int64_t(c) * g.Np;
    T* tho = theta_out + int64_t(c) * g.Np;
    const T* fc = f ? f + int64_t(c) * fcs : nullptr;
    // Tile load in chunks of KB entries per thread: the loads of a chunk are
    // branch-free (positions outside the grid read offset 0 of the field,
    // which is padding and stays zero; the prolongation reads clamped nodes
    // and is masked), so they are all in flight before the LDS writes.
    constexpr int KF = (RX * RY + kBlock - 1) / kBlock, KB = PROLONG ? 2 : 4;
#pragma unroll 1
    for (int k0 = 0; k0 < KF; k0 += KB) {
      T v[KB];
#pragma unroll
      for (int u = 0; u < KB; ++u) {
        const int idx = min(int(threadIdx.x) + (k0 + u) * kBlock, RX * RY - 1);
        const int x = ox + idx % RX, y = oy + idx / RX;
        const bool in = x >= 1 && x <= n && y >= 1 && y <= n;
        T a = thi[(in && !zero_in) ? pidx(g, x, y, 0) : 0];
        if (PROLONG) {
          const int xc = min(max(x, 1), n), yc = min(max(y, 1), n);
          const T pr = prolong_at<T, USERP>(psi + int64_t(c) * gc.Np, gc, wP, xc, yc);
          a += in ? pr : T(0);
        }
        v[u] = a;
      }
#pragma unroll
      for (int u = 0; u < KB; ++u) {
        const int idx = int(threadIdx.x) + (k0 + u) * kBlock;
        if (idx < RX * RY) sh[Z::pos(idx % RX, idx / RX)] = v[u];
      }
    }
    __syncthreads();
    for (int p = 0; p < NPASS; ++p) {
      const int pos = backward ? NPASS - 1 - p : p;  // position in the forward order
      const int hp = NPASS - 1 - p;
      const int xlo = max(1, tx0 - hp), xhi = min(n, tx0 + TX - 1 + hp);
      const int ylo = max(1, ty0 - hp), yhi = min(n, ty0 + TY - 1 + hp);
      const int nrows = yhi - ylo + 1;
      if (xlo <= xhi && nrows > 0) {
        for (int item = threadIdx.x; item < nrows * Q; item += blockDim.x) {
          const int y = ylo + item / Q;
          const int qi = item % Q;
          int colour;
          if (NPASS == 2) {
            const int ypar = y & 1;
            const int xpar = (pos == 0) ? ypar : 1 - ypar;  // red (equal parities) first
            colour = xpar | (ypar << 1);
          } else {
            colour = kFwdOrder2[pos];
            if (((colour >> 1) & 1) != (y & 1)) continue;
          }
          const int xpar = colour & 1;
          const int off = xpar ? 1 : 2;
          const int q = (xlo - off + 5) / 4 - 1 + qi;  // first pair whose second site >= xlo
          const int xa = 4 * q + off;
          if (xa > xhi) continue;
          // Issue every global load of the pair first (addresses clamped into the
          // pass region so the loads are unconditional); the Philox and
          // Box-Muller arithmetic below then hides their latency.
          constexpr int NB = CROSS ? 4 : 8;
          T cf[2][NB], rhs[2], ivd[2], isd[2];
          int64_t gi[2];
          int li[2];
          bool live[2];
#pragma unroll
          for (int k = 0; k < 2; ++k) {
            const int x = xa + 2 * k;
            live[k] = x >= xlo && x <= xhi;
            const int xc = min(max(x, xlo), xhi);
            gi[k] = pidx(g, xc, y, 0);
            li[k] = Z::pos(xc - ox, y - oy);
            rhs[k] = fc ? fc[gi[k]] : T(0);
            int b = 0;
#pragma unroll
            for (int t = 0; t < 9; ++t) {
              const int dx = t % 3 - 1, dy = t / 3 - 1;
              if (dx == 0 && dy == 0) continue;
              if (CROSS && dx != 0 && dy != 0) continue;
              cf[k][b++] = stencil_entry<T, 2>(coef, g, t, gi[k]);
            }
            ivd[k] = invd[gi[k]];
            isd[k] = isqd[gi[k]];
          }
          const int m1 = xpar ? (n + 1) / 2 : (n - 1) / 2;
          const int qx = (m1 + 1) / 2;
          const uint32_t pair = uint32_t(q) + uint32_t(qx) * uint32_t((y - 1) >> 1);
          const Block4 blk = philox10(pair, word | uint32_t(colour), m, 0u, seed, chain0 + c);
          T z[2];
          Gauss<T>::pair(blk, z[0], z[1]);
          // the two sites are two apart in x, so they sit in different sub-rows
#pragma unroll
          for (int k = 0; k < 2; ++k) {
            if (!live[k]) continue;
            const int sx = (xa + 2 * k - ox) & 3;
            const int oe = Z::east(sx), ow = Z::west(sx);
            T s = rhs[k];
            int b = 0;
#pragma unroll
            for (int t = 0; t < 9; ++t) {
              const int dx = t % 3 - 1, dy = t / 3 - 1;
              if (dx == 0 && dy == 0) continue;
              if (CROSS && dx != 0 && dy != 0) continue;
              const int o = dy * Z::RS + (dx < 0 ? ow : (dx > 0 ? oe : 0));
              s -= cf[k][b++] * sh[li[k] + o];
            }
            sh[li[k]] = s * ivd[k] + z[k] * isd[k];
          }
        }
      }
      __syncthreads();
    }
    if (bs.snap) snap_sites(bs, g, int(blockIdx.x), c, ox, oy, int(blockDim.x),
                            [&](int lx, int ly) { return double(sh[Z::pos(lx, ly)]); });
    for (int idx = threadIdx.x; idx < TX * TY; idx += blockDim.x) {
      const int x = tx0 + idx % TX, y = ty0 + idx / TX;
      if (x <= n && y <= n) tho[pidx(g, x, y, 0)] = sh[Z::pos(x - ox, y - oy)];
    }
    __syncthreads();
  }
}

// Segment form of the tiled sweep.  Thread (sy, sx) owns the four sites
// x = 4q+1 .. 4q+4 of one row; such a segment holds exactly one Philox pair
// of each colour present in its row.  The thread loads its segment's stencil
// (and the shared right-hand side) once per block into registers with
// contiguous loads, and reuses them for every colour pass and every chain of
// the block; only the states go through LDS.  Rows cover the tile plus
// NPASS-1 halo rows, segments the tile plus one segment either side.
//
// With DMA (5-point levels) the state region and coarse patch of each chain
// travel from memory straight into an LDS staging buffer (global_load_lds,
// 16 contiguous bytes per lane), one of two: the next chain's copy is issued
// when the current chain starts its colour passes, so it is in flight while
// they run, and costs no registers.  Each chain then moves its staging into
// the tile layout, adding the prolongation on the way.
template <typename T, int NPASS, bool PROLONG, bool USERP, int TYS, int NT, int MC, bool DMA>
__global__ __launch_bounds__(NT) void k_sweep2d_seg(
    const T* __restrict__ coef, const T* __restrict__ invd, const T* __restrict__ isqd,
    const T* __restrict__ theta_in, T* __restrict__ theta_out, int zero_in,
    const T* __restrict__ f, int64_t fcs, Geom g,
    const T* __restrict__ psi, Geom gc, const double* __restrict__ wP, int backward,
    uint32_t word, const int64_t* __restrict__ mcur, uint32_t seed, uint32_t chain0, int tiles_x,
    int cpb, int nchains, const double* __restrict__ bmtab, BSnap bs) {
  constexpr bool CROSS = (NPASS == 2);
  constexpr int TX = 64, SX = TX / 4 + 2;       // segments per row (tile + one each side)
  constexpr int SY = TYS + 2 * (NPASS - 1);     // rows with owners
  constexpr int HALF = SY / 2;                  // rows of each parity
  constexpr int GA = (HALF * SX + 63) / 64 * 64;  // threads of the first parity group
  constexpr int H = NPASS, RX = TX + 2 * H, RY = TYS + 2 * H;
  constexpr int NB = CROSS ? 4 : 8;
  // right-hand side: shared by all chains (or absent) on the 5-point finest
  // level, one per chain on the 9-point coarse levels
  constexpr bool RHSC = !CROSS;
  static_assert(SY % 2 == 0, "owner rows must split evenly by parity");
  static_assert(GA + HALF * SX <= NT, "block too small for the segment grid");
  using Z = Swz<RX, int(sizeof(T))>;
  __shared__ T sh[DMA ? 1 : MC][DMA ? 1 : RY * Z::RS];
  // coarse patch under the tile region for the fused prolongation
  constexpr int CRX = RX / 2 + 2, CRY = RY / 2 + 2;
  constexpr int KP = PROLONG ? (CRX * CRY + NT - 1) / NT : 0;
  __shared__ T spsi[DMA ? 1 : MC][PROLONG && !DMA ? CRY * CRX : 1];
  // DMA staging (two buffers per array): rows of the region as they lie in
  // memory, in 16-byte chunks from the aligned element SH0 places left of
  // the region's first column (each region row starts 2 elements past a
  // 16-byte boundary of the padded layout)
  constexpr int CH = 16 / int(sizeof(T));  // elements per chunk
  constexpr int SH0 = 2 % CH;
  constexpr int NCT = (RX + SH0 + CH - 1) / CH, NCP = (CRX + SH0 + CH - 1) / CH;  // chunks per row
  constexpr int RST = NCT * CH, RSP = NCP * CH;                                 // row pitches
  __shared__ __attribute__((aligned(16))) T stA[DMA ? RY * RST : 1], stB[DMA ? RY * RST : 1];
  __shared__ T shT[DMA ? RY * Z::RS : 1];  // the tile in layout Z
  __shared__ __attribute__((aligned(16))) T spA[DMA && PROLONG ? CRY * RSP : 1],
      spB[DMA && PROLONG ? CRY * RSP : 1];
  static_assert(!DMA || (MC == 1 && CROSS), "LDS DMA tiles: 5-point levels, one chain per step");
  // double precision draws its normals with the table-driven Box-Muller;
  // the table's loads are issued first and written to LDS only after the
  // stencil loads below are in flight too
  constexpr bool TAB = sizeof(T) == 8;
  constexpr int KTAB = TAB ? (kBmTable + NT - 1) / NT : 1;
  __shared__ double stab[TAB ? kBmTable : 1];
  double tabv[KTAB];
  if (TAB) {
#pragma unroll
    for (int k = 0; k < KTAB; ++k) tabv[k] = bmtab[min(int(threadIdx.x) + k * NT, kBmTable - 1)];
  }
  const int n = g.n;
  const int tx0 = int(blockIdx.x % tiles_x) * TX + 1;
  const int ty0 = int(blockIdx.x / tiles_x) * TYS + 1;
  const int ox = tx0 - H, oy = ty0 - H;
  const uint32_t m = uint32_t(*mcur);
  // Owners grouped by row parity (each group starts on a wavefront boundary)
  // so that every wavefront updates a single colour in each pass.
  const int y0 = ty0 - (NPASS - 1);
  const int grp = int(threadIdx.x) < GA ? 0 : 1;
  const int u = int(threadIdx.x) - grp * GA;
  const int sx = u % SX, srow = u / SX;
  const bool owner = srow < HALF;
  const int par0 = (y0 & 1);  // row offset of the group whose rows are even
  const int r = 2 * srow + (grp == 0 ? par0 : 1 - par0);
  const int q = (tx0 - 1) / 4 - 1 + sx;  // segment index: sites 4q+1 .. 4q+4
  const int y = y0 + r;
  const bool row_in = owner && y >= 1 && y <= n;
  // stencil of the four sites in registers (zero outside the grid)
  T cf[4][NB], ivd[4], isd[4], rhs[RHSC ? 1 : 4];
  if (CROSS) {
    // The 5-point operator is symmetric entry by entry (east of x is west of
    // x + 1, north of y is south of y + 1), so only the west and south arrays
    // are read: five west entries and the south entries of rows y and y + 1.
    T wv[5], sv[4], nv[4];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const int x = 4 * q + 1 + k;
      const bool in = row_in && x >= 1 && x <= n;
      wv[k] = coef[int64_t(3) * g.Np + (in ? pidx(g, x, y, 0) : 0)];
      if (k < 4) {
        sv[k] = coef[int64_t(1) * g.Np + (in ? pidx(g, x, y, 0) : 0)];
        nv[k] = coef[int64_t(1) * g.Np + ((in && y + 1 <= n) ? pidx(g, x, y + 1, 0) : 0)];
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      cf[k][0] = sv[k];      // (0, -1)
      cf[k][1] = wv[k];      // (-1, 0)
      cf[k][2] = wv[k + 1];  // (+1, 0)
      cf[k][3] = nv[k];      // (0, +1)
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int x = 4 * q + 1 + k;
    const bool in = row_in && x >= 1 && x <= n;
    const int64_t gi = in ? pidx(g, x, y, 0) : 0;
    if (!CROSS) {
      // entries towards +x / +y from the neighbour's opposite entry (the
      // operator is symmetric entry by entry), so four of the eight
      // neighbour arrays are read
      int b = 0;
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        const int dx = t % 3 - 1, dy = t / 3 - 1;
        if (dx == 0 && dy == 0) continue;
        const bool mirror = t > 4;
        const int64_t at = mirror ? (in ? pidx(g, x + dx, y + dy, 0) : 0) : gi;
        cf[k][b++] = coef[int64_t(mirror ? 8 - t : t) * g.Np + at];
      }
    }
    ivd[k] = invd[gi];
    isd[k] = sqrt(ivd[k]);  // A_ii^{-1/2} as sqrt(1 / A_ii): one array fewer to read
    if (!RHSC) rhs[k] = f ? f[gi] : T(0);
  }
  // The passes this thread updates sites in ("slots"): on red-black levels
  // both passes (each row holds both colours), on four-colour levels the
  // two passes whose colours live on rows of this thread's parity.
  auto pass_colour = [&](int p) -> int {
    const int pos = backward ? NPASS - 1 - p : p;
    if (NPASS == 2) {
      const int ypar = y & 1;
      return (pos == 0 ? ypar : 1 - ypar) | (ypar << 1);
    }
    return kFwdOrder2[pos];
  };
  auto pass_active = [&](int p) -> bool {
    const int hp = NPASS - 1 - p;
    return row_in && y >= ty0 - hp && y <= ty0 + TYS - 1 + hp &&
           (NPASS == 2 || ((pass_colour(p) >> 1) & 1) == (y & 1));
  };
  int pslot[2];
  if (NPASS == 2) {
    pslot[0] = 0;
    pslot[1] = 1;
  } else {  // forward positions of colours {0, 1} (even rows) or {3, 2} (odd rows)
    const int pos0 = (y & 1) ? 1 : 0, pos1 = pos0 + 2;
    pslot[0] = backward ? NPASS - 1 - pos0 : pos0;
    pslot[1] = backward ? NPASS - 1 - pos1 : pos1;
  }
  constexpr bool HOIST = CROSS || !PROLONG || sizeof(T) == 4;
  constexpr bool AHEAD = NPASS == 4 && MC == 1;  // normals drawn in the idle pass before
  const int cb = int(blockIdx.y) * cpb;
  const int ce = min(nchains, cb + cpb);
  const int jx0 = ox >> 1, jy0 = oy >> 1;  // first coarse node under the region
  auto draw = [&](int c, int p, T& z0, T& z1) {
    const int colour = pass_colour(p);
    const int xpar = colour & 1;
    const int m1 = xpar ? (n + 1) / 2 : (n - 1) / 2;
    const int qx = (m1 + 1) / 2;
    const uint32_t pair = uint32_t(q) + uint32_t(qx) * uint32_t((y - 1) >> 1);
    const Block4 blk = philox10(pair, word | uint32_t(colour), m, 0u, seed, chain0 + c);
    if constexpr (TAB) {
      double a0, a1;
      gauss_pair_tab(blk, stab, a0, a1);
      z0 = T(a0);
      z1 = T(a1);
    } else {
      Gauss<T>::pair(blk, z0, z1);
    }
  };
  // colour pass p of one chain on the LDS tile s: the thread's sites of
  // that colour (z0, z1: their normals; rcv: the chain's right-hand side on
  // 9-point levels)
  auto pass_update = [&](int p, T* s, T z0, T z1, const T* rcv) __attribute__((always_inline)) {
    const int hp = NPASS - 1 - p;
    const int colour = pass_colour(p);
    const int xpar = colour & 1;
    const int k0 = xpar ? 0 : 1;  // offset of the colour's first site in the segment
    const int xlo = max(1, tx0 - hp), xhi = min(n, tx0 + TX - 1 + hp);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
#pragma unroll
      for (int kk = 0; kk < 2; ++kk) {  // resolve the site index at compile time
        if (kk != k0) continue;
        const int k = kk + 2 * j;
        const int x = 4 * q + 1 + k;
        if (x < xlo || x > xhi) continue;
        const int lx = x - ox;
        // lx = x - tx0 + H with x = 4 q + 1 + k and tx0 = 1 (mod 4), so the
        // sub-row lx & 3 is known at compile time (constant LDS offsets)
        const int sxm = (k + H) & 3;
        const int li = (y - oy) * Z::RS + sxm * Z::W + (lx >> 2);
        const int oe = Z::east(sxm), ow = Z::west(sxm);
        T sum = RHSC ? rcv[k] : rhs[RHSC ? 0 : k];
        int b = 0;
#pragma unroll
        for (int t = 0; t < 9; ++t) {
          const int dx = t % 3 - 1, dy = t / 3 - 1;
          if (dx == 0 && dy == 0) continue;
          if (CROSS && dx != 0 && dy != 0) continue;
          const int o = dy * Z::RS + (dx < 0 ? ow : (dx > 0 ? oe : 0));
          sum -= cf[k][b++] * s[li + o];
        }
        // one explicit contraction, the same in every form that inlines this
        s[li] = fma(sum, ivd[k], (j == 0 ? z0 : z1) * isd[k]);
      }
    }
  };
  // The tile's snapshot slots (the same for every chain): thread t keeps
  // slot b0 + t and its LDS position, so that no chain loads the lists
  // again; slots past b0 + NT (rare) are looked up per chain.
  int snap_slot = -1, snap_pos = 0, snap_b0 = 0, snap_b1 = 0;
  double snap_w = 0.0;
  if (bs.snap) {
    snap_b0 = bs.ptr[blockIdx.x];
    snap_b1 = bs.ptr[blockIdx.x + 1];
    if (snap_b0 + int(threadIdx.x) < snap_b1) {
      snap_slot = bs.ent[snap_b0 + int(threadIdx.x)];
      const int site = bs.idx[snap_slot];
      snap_pos = Z::pos(site % g.px - 3 - ox, site / g.px - oy);
      snap_w = bs.w[snap_slot];
    }
  }
  // snapshot of B's sites (weight times value) and the tile's output of
  // chain c from LDS tile s
  auto finish_chain = [&](int c, const T* s) __attribute__((always_inline)) {
    if (snap_slot >= 0) bs.snap[int64_t(c) * bs.nnz + snap_slot] = snap_w * double(s[snap_pos]);
    for (int i = snap_b0 + NT + int(threadIdx.x); i < snap_b1; i += NT) {
      const int e = bs.ent[i];
      const int site = bs.idx[e];
      bs.snap[int64_t(c) * bs.nnz + e] = bs.w[e] * double(s[Z::pos(site % g.px - 3 - ox, site / g.px - oy)]);
    }
    if (row_in && sx >= 1 && sx <= TX / 4 && y >= ty0 && y <= ty0 + TYS - 1) {
      T* tho = theta_out + int64_t(c) * g.Np;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int x = 4 * q + 1 + k;
        if (x <= n) tho[pidx(g, x, y, 0)] = s[Z::pos(x - ox, y - oy)];
      }
    }
  };
  constexpr int KF = (RX * RY + NT - 1) / NT;  // tile elements per thread
  if (TAB) {
#pragma unroll
    for (int k = 0; k < KTAB; ++k)
      if (int(threadIdx.x) + k * NT < kBmTable) stab[int(threadIdx.x) + k * NT] = tabv[k];
    __syncthreads();
  }
  if constexpr (DMA) {
    const int tid = int(threadIdx.x);
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    // LDS DMA of chain c's state region into dst (and coarse patch into
    // dsp), one 16-byte chunk per lane: instruction k fills chunks
    // 64 k .. 64 k + 63 of the staging buffer, row by row.  A chunk of a row
    // outside the grid, or starting right of it, reads offset 0 of the field
    // (padding, zero); other chunks read memory as it lies, where the
    // columns outside the grid are ghost entries (zero).
    auto dma = [&](int c, T* dst, T* dsp) __attribute__((always_inline)) {
      const T* thi = theta_in + int64_t(c) * g.Np;
      for (int k = wave; k < (RY * NCT + 63) / 64; k += NT / 64) {
        const int d = k * 64 + lane, ly = d / NCT, xf = ox - SH0 + (d % NCT) * CH;
        const int yy = oy + ly;
        const bool ok = !zero_in && d < RY * NCT && yy >= 1 && yy <= n && xf <= n;
        if (d < RY * NCT)
          lds_dma16(thi + (ok ? pidx(g, xf, yy, 0) : 0), dst + k * 64 * CH);
      }
      if (PROLONG) {
        const T* ps = psi + int64_t(c) * gc.Np;
        for (int k = wave; k < (CRY * NCP + 63) / 64; k += NT / 64) {
          const int d = k * 64 + lane, r = d / NCP, jf = jx0 - SH0 + (d % NCP) * CH;
          const int Jy = jy0 + r;
          const bool ok = d < CRY * NCP && Jy >= 1 && Jy <= gc.n && jf <= gc.n;
          if (d < CRY * NCP)
            lds_dma16(ps + (ok ? pidx(gc, jf, Jy, 0) : 0), dsp + k * 64 * CH);
        }
      }
    };
    auto chain = [&](int c, const T* cst, const T* csp, T* nst, T* nsp) __attribute__((always_inline)) {
      // this chain's staging has landed (and the previous chain's stores are done)
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      // staging -> tile layout Z, with the prolongation added
#pragma unroll
      for (int k = 0; k < KF; ++k) {
        const int idx = tid + k * NT;
        if (idx >= RX * RY) continue;
        const int lx = idx % RX, ly = idx / RX;
        T v = cst[ly * RST + SH0 + lx];
        const int xx = ox + lx, yy = oy + ly;
        if (PROLONG && xx >= 1 && xx <= n && yy >= 1 && yy <= n)
          v += prolong_lds<T, USERP>(csp + SH0, RSP, jx0, jy0, gc, wP, xx, yy);
        shT[Z::pos(lx, ly)] = v;
      }
      __syncthreads();
      if (c + 1 < ce) dma(c + 1, nst, nsp);
      T zz[2][2];
#pragma unroll
      for (int sl = 0; sl < 2; ++sl) {
        zz[sl][0] = zz[sl][1] = T(0);
        if (HOIST && pass_active(pslot[sl])) draw(c, pslot[sl], zz[sl][0], zz[sl][1]);
      }
#pragma unroll
      for (int p = 0; p < NPASS; ++p) {
        if ((p == pslot[0] || p == pslot[1]) && pass_active(p)) {
          T z0 = p == pslot[0] ? zz[0][0] : zz[1][0];
          T z1 = p == pslot[0] ? zz[0][1] : zz[1][1];
          if (!HOIST) draw(c, p, z0, z1);
          pass_update(p, shT, z0, z1, nullptr);
        }
        lds_barrier();
      }
      finish_chain(c, shT);
    };
    if (cb < ce) dma(cb, stA, spA);
    for (int c = cb; c < ce; c += 2) {
      chain(c, stA, spA, stB, spB);
      if (c + 1 < ce) chain(c + 1, stB, spB, stA, spA);
    }
    return;
  }
  // MC chains per step: their tiles sit side by side in LDS and every pass
  // updates all of them between two barriers.  A step past the last chain
  // works on the last chain's data and stores nothing.
  for (int c0 = cb; c0 < ce; c0 += MC) {
    const int tid = int(threadIdx.x);
    // Every load below is issued unconditionally: positions outside the grid
    // (or all of them when the input is zero) read offset 0 of the field,
    // which is padding and stays zero.  Without per-load branches the loaded
    // registers need no copies, so nothing waits for the loads before the
    // noise below is drawn.
    T rc[RHSC ? MC : 1][4], pv[MC][KP > 0 ? KP : 1], fv[MC][KF];
#pragma unroll
    for (int mi = 0; mi < MC; ++mi) {
      const int c = min(c0 + mi, ce - 1);
      if (RHSC) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int x = 4 * q + 1 + k;
          rc[mi][k] = f[int64_t(c) * fcs + ((row_in && x >= 1 && x <= n) ? pidx(g, x, y, 0) : 0)];
        }
      }
#pragma unroll
      for (int k = 0; k < KP; ++k) {
        const int e = tid + k * NT;
        const int Jx = jx0 + e % CRX, Jy = jy0 + e / CRX;
        const bool ok = e < CRX * CRY && Jx >= 1 && Jx <= gc.n && Jy >= 1 && Jy <= gc.n;
        pv[mi][k] = psi[int64_t(c) * gc.Np + (ok ? pidx(gc, Jx, Jy, 0) : 0)];
      }
      const T* thi = theta_in + int64_t(c) * g.Np;
#pragma unroll
      for (int k = 0; k < KF; ++k) {
        const int idx = tid + k * NT;
        const int xx = ox + idx % RX, yy = oy + idx / RX;
        const bool ok = !zero_in && idx < RX * RY && xx >= 1 && xx <= n && yy >= 1 && yy <= n;
        fv[mi][k] = thi[ok ? pidx(g, xx, yy, 0) : 0];
      }
    }
    // ... and draw the noise while they are in flight (except where
    // registers are scarce: FP64 four-colour levels with the prolongation)
    // (on four-colour levels with one chain per step, only a draw for pass
    // 0; the others come during the idle pass before theirs, below)
    T zz[MC][2][2];
#pragma unroll
    for (int mi = 0; mi < MC; ++mi) {
#pragma unroll
      for (int sl = 0; sl < 2; ++sl) {
        zz[mi][sl][0] = zz[mi][sl][1] = T(0);
        if (HOIST && (!AHEAD || pslot[sl] == 0) && c0 + mi < ce && pass_active(pslot[sl]))
          draw(c0 + mi, pslot[sl], zz[mi][sl][0], zz[mi][sl][1]);
      }
    }
    if (PROLONG) {
#pragma unroll
      for (int mi = 0; mi < MC; ++mi) {
#pragma unroll
        for (int k = 0; k < KP; ++k) {
          const int e = tid + k * NT;
          if (e < CRX * CRY) spsi[mi][e] = pv[mi][k];
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int mi = 0; mi < MC; ++mi) {
#pragma unroll
      for (int k = 0; k < KF; ++k) {
        const int idx = tid + k * NT;
        if (idx >= RX * RY) continue;
        const int xx = ox + idx % RX, yy = oy + idx / RX;
        T v = fv[mi][k];
        if (PROLONG && xx >= 1 && xx <= n && yy >= 1 && yy <= n)
          v += prolong_lds<T, USERP>(spsi[mi], CRX, jx0, jy0, gc, wP, xx, yy);
        sh[mi][Z::pos(idx % RX, idx / RX)] = v;
      }
    }
    __syncthreads();
    // On four-colour levels with one chain per step a thread draws the
    // normals of its next pass during the pass before it, in which its rows
    // have no colour to update (its two passes have one parity); only pass
    // 0 takes normals drawn before the passes (hoisted) or in place.
    T za0 = T(0), za1 = T(0);
#pragma unroll
    for (int p = 0; p < NPASS; ++p) {
      if ((p == pslot[0] || p == pslot[1]) && pass_active(p)) {
#pragma unroll
        for (int mi = 0; mi < MC; ++mi) {
          T z[2] = {p == pslot[0] ? zz[mi][0][0] : zz[mi][1][0],
                    p == pslot[0] ? zz[mi][0][1] : zz[mi][1][1]};
          if (AHEAD && p > 0) {
            z[0] = za0;
            z[1] = za1;
          } else if (!HOIST) {
            draw(min(c0 + mi, ce - 1), p, z[0], z[1]);
          }
          pass_update(p, sh[mi], z[0], z[1], rc[RHSC ? mi : 0]);
        }
      } else if (AHEAD && p + 1 < NPASS && (p + 1 == pslot[0] || p + 1 == pslot[1]) &&
                 pass_active(p + 1)) {
        draw(c0, p + 1, za0, za1);
      }
      __syncthreads();
    }
#pragma unroll
    for (int mi = 0; mi < MC; ++mi) {
      const int c = c0 + mi;
      if (c >= ce) break;
      finish_chain(c, sh[mi]);
    }
    __syncthreads();
  }
}


// The same restriction with the residual's operator held in registers across
// the chains of a block.  A block covers CTX x CTY coarse nodes; thread t
// owns the fine residual nodes t, t + NT, ... of the (2 CTX + 1) x (2 CTY + 1)
// residual region and keeps their stencil (and a chain-shared right-hand
// side) in registers.  Per chain: the theta region (one more ring) goes from
// registers to LDS, each thread forms its residuals into LDS, and thread J
// sums the nine weighted residuals of coarse node J.  The next chain's theta
// (and right-hand side) loads are issued before the current chain's
// residuals, and every load is branch-free: positions outside the grid read
// offset 0 of the field, which is padding and stays zero.
template <typename T, bool CROSS, bool USERP, int CTY, int NT>
__global__ __launch_bounds__(NT) void k_restrict2d_reg(
    const T* __restrict__ coef, const T* __restrict__ theta, const T* __restrict__ f, int64_t fcs,
    Geom gf, T* __restrict__ fcoarse, Geom gc, const double* __restrict__ wP, int tiles_x, int cpb,
    int nchains, LowRankRhs lr) {
  constexpr int CTX = 32;
  constexpr int RXr = 2 * CTX + 1, RYr = 2 * CTY + 1;  // residual region
  constexpr int RXt = RXr + 2, RYt = RYr + 2;          // theta region
  constexpr int KR = (RXr * RYr + NT - 1) / NT;        // residual nodes per thread
  constexpr int KT = (RXt * RYt + NT - 1) / NT;        // theta entries per thread
  constexpr int NS = CROSS ? 5 : 9;
  static_assert(CTX * CTY <= NT, "one coarse node per thread");
  __shared__ T sth[RYt * RXt];
  __shared__ T sr[RYr * RXr];
  const int nf = gf.n, nc = gc.n;
  const int cx0 = int(blockIdx.x % tiles_x) * CTX + 1;
  const int cy0 = int(blockIdx.x / tiles_x) * CTY + 1;
  const int rx0 = 2 * cx0 - 1, ry0 = 2 * cy0 - 1;
  const int tx0 = rx0 - 1, ty0 = ry0 - 1;
  const int tid = int(threadIdx.x);
  // stencil of the owned residual nodes (zero outside the grid)
  int64_t gr[KR];
  T cr[KR][NS], fr[KR];
#pragma unroll
  for (int k = 0; k < KR; ++k) {
    const int idx = tid + k * NT;
    const int x = rx0 + idx % RXr, y = ry0 + idx / RXr;
    const bool in = idx < RXr * RYr && x >= 1 && x <= nf && y >= 1 && y <= nf;
    gr[k] = in ? pidx(gf, x, y, 0) : 0;
    int b = 0;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int dx = t % 3 - 1, dy = t / 3 - 1;
      if (CROSS && dx != 0 && dy != 0) continue;
      // The operator is symmetric entry by entry: an entry towards +x or +y
      // is the opposite entry of that neighbour, so only the centre and the
      // entries towards -x / -y are read from memory.  (Next to the boundary
      // the neighbour is a ghost entry, zero, and so is the state it meets.)
      const bool mirror = t > 4;
      const int64_t at = mirror ? (in ? pidx(gf, x + dx, y + dy, 0) : 0) : gr[k];
      cr[k][b++] = coef[int64_t(mirror ? 8 - t : t) * gf.Np + at];
    }
    fr[k] = (f && fcs == 0) ? f[gr[k]] : T(0);
  }
  // this thread's coarse node
  const int J1 = cx0 + tid % CTX, J2 = cy0 + tid / CTX;
  const bool own = tid < CTX * CTY && J1 <= nc && J2 <= nc;
  const int64_t iJ = own ? pidx(gc, J1, J2, 0) : 0;
  const int rowJ = (own && lr.row_of) ? lr.row_of[iJ] : -1;
  T wJ[9];
#pragma unroll
  for (int t1 = 0; t1 < 9; ++t1) {
    const int ex = t1 % 3 - 1, ey = t1 / 3 - 1;
    wJ[t1] = USERP ? T(wP[int64_t(t1) * gc.Np + iJ]) : T(multilinear(ex, ey, 0));
  }
  const int cb = int(blockIdx.y) * cpb;
  const int ce = min(nchains, cb + cpb);
  T tv[KT], fn[KR];
  auto issue = [&](int c) {
    const T* th = theta + int64_t(c) * gf.Np;
#pragma unroll
    for (int k = 0; k < KT; ++k) {
      const int idx = tid + k * NT;
      const int x = tx0 + idx % RXt, y = ty0 + idx / RXt;
      const bool ok = idx < RXt * RYt && x >= 1 && x <= nf && y >= 1 && y <= nf;
      tv[k] = th[ok ? pidx(gf, x, y, 0) : 0];
    }
    if (f && fcs != 0) {
#pragma unroll
      for (int k = 0; k < KR; ++k) fn[k] = f[int64_t(c) * fcs + gr[k]];
    }
  };
  if (cb < ce) issue(cb);
  for (int c = cb; c < ce; ++c) {
#pragma unroll
    for (int k = 0; k < KT; ++k) {
      const int idx = tid + k * NT;
      if (idx < RXt * RYt) sth[idx] = tv[k];
    }
    if (f && fcs != 0) {
#pragma unroll
      for (int k = 0; k < KR; ++k) fr[k] = fn[k];
    }
    __syncthreads();
    if (c + 1 < ce) issue(c + 1);
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      const int idx = tid + k * NT;
      if (idx >= RXr * RYr) continue;
      const int lx = idx % RXr, ly = idx / RXr;
      const int li = (ly + 1) * RXt + (lx + 1);
      T r = fr[k];
      int b = 0;
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        const int dx = t % 3 - 1, dy = t / 3 - 1;
        if (CROSS && dx != 0 && dy != 0) continue;
        r -= cr[k][b++] * sth[li + dy * RXt + dx];
      }
      sr[idx] = r;
    }
    __syncthreads();
    if (own) {
      const int lx = 2 * (J1 - cx0) + 1, ly = 2 * (J2 - cy0) + 1;
      T acc = T(0);
#pragma unroll
      for (int t1 = 0; t1 < 9; ++t1) {
        const int ex = t1 % 3 - 1, ey = t1 / 3 - 1;
        acc += wJ[t1] * sr[(ly + ey) * RXr + (lx + ex)];
      }
      double lrv = 0.0;
      if (rowJ >= 0) {
        for (int64_t e = lr.ptr[rowJ]; e < lr.ptr[rowJ + 1]; ++e)
          lrv += lr.val[e] * lr.v[int64_t(c) * lr.beta + lr.col[e]];
      }
      fcoarse[int64_t(c) * gc.Np + iJ] = T(double(acc) - lrv);
    }
    __syncthreads();
  }
}

constexpr int kTX = 64, kTY = 32;  // sweep tile

int chains_per_block(int nchains, int64_t tiles) {
  // enough blocks to cover the 256 compute units several times over, while
  // keeping chains together so the operator stays cache-resident
  int64_t cpb = (int64_t(nchains) * tiles) / 2048;
  if (cpb < 1) cpb = 1;
  if (cpb > nchains) cpb = nchains;
  return int(cpb);
}

}  // namespace

void fill_bm_table(double* t) {
  const long double two_pi = 6.283185307179586476925286766559005768L;
  for (int i = 0; i < 128; ++i) {
    const long double c = 45.0L / 64.0L + (i + 0.5L) * (45.0L / 8192.0L);
    t[i] = double(std::log(c));
    t[128 + i] = double(1.0L / c);
  }
  for (int k = 0; k <= 256; ++k) {
    long double sn = std::sin(two_pi * k / 256.0L), cs = std::cos(two_pi * k / 256.0L);
    if (k % 64 == 0) {  // exact on the axes
      const int q = k / 64;
      sn = (q == 1) ? 1.0L : (q == 3 ? -1.0L : 0.0L);
      cs = (q == 0 || q == 4) ? 1.0L : (q == 2 ? -1.0L : 0.0L);
    }
    t[256 + k] = double(sn);
    t[513 + k] = double(cs);
  }
}

// The snapshot of B's sites for the fused low-rank step (fixed-width slots
// per column of B), in the slot lists of tile height index gi.
static BSnap make_snap(const DevLevel& lv, int gi, bool snap) {
  BSnap bs;
  if (!snap) return bs;
  bs.ptr = lv.bt_ptr[gi];
  bs.ent = lv.bt_ent[gi];
  bs.idx = lv.bpidx;
  bs.w = lv.bpval;
  bs.snap = lv.bsnap;
  bs.nnz = lv.bslots;
  return bs;
}

hipError_t launch_sweep_tiled(const Launch& L, const DevLevel& lv, const void* theta_in,
                              void* theta_out, int zero_in, const void* f, int64_t fcs,
                              uint32_t word, int backward, const DevLevel* coarse, const void* psi,
                              bool snap) {
  if (L.mcur == nullptr || L.dim != 2 || theta_in == theta_out) return hipErrorInvalidValue;
  if (coarse != nullptr && psi == nullptr) return hipErrorInvalidValue;
  if (snap && (lv.bsnap == nullptr || lv.bt_ptr[0] == nullptr)) return hipErrorInvalidValue;
  const BSnap bs = make_snap(lv, 0, snap);
  const int n = lv.g.n;
  const int tiles_x = (n + kTX - 1) / kTX, tiles_y = (n + kTY - 1) / kTY;
  const int64_t tiles = int64_t(tiles_x) * tiles_y;
  const int cpb = chains_per_block(L.nchains, tiles);
  dim3 grid(unsigned(tiles), unsigned((L.nchains + cpb - 1) / cpb));
  const bool pro = coarse != nullptr;
  const bool userp = pro && lv.wP != nullptr;
  const Geom gc = pro ? coarse->g : Geom{};
#define MGMC_SWEEP_T(T, NP, PR, UP)                                                                  \
  k_sweep2d_tiled<T, NP, PR, UP, kTX, kTY><<<grid, kBlock, 0, L.stream>>>(                          \
      (const T*)lv.coef, (const T*)lv.invd, (const T*)lv.isqd, (const T*)theta_in, (T*)theta_out,     \
      zero_in, (const T*)f, fcs, lv.g, (const T*)psi, gc, userp ? lv.wP : nullptr, backward, word,     \
      L.mcur,                                                                                          \
      L.seed, L.chain0, tiles_x, cpb, L.nchains, bs)
#define MGMC_SWEEP_NP(T, NP)                      \
  do {                                            \
    if (!pro) MGMC_SWEEP_T(T, NP, false, false);  \
    else if (!userp) MGMC_SWEEP_T(T, NP, true, false); \
    else MGMC_SWEEP_T(T, NP, true, true);         \
  } while (0)
  if (L.fp32) {
    if (lv.cross) MGMC_SWEEP_NP(float, 2); else MGMC_SWEEP_NP(float, 4);
  } else {
    if (lv.cross) MGMC_SWEEP_NP(double, 2); else MGMC_SWEEP_NP(double, 4);
  }
#undef MGMC_SWEEP_NP
#undef MGMC_SWEEP_T
  return hipGetLastError();
}

hipError_t launch_sweep_seg(const Launch& L, const DevLevel& lv, const void* theta_in,
                            void* theta_out, int zero_in, const void* f, int64_t fcs,
                            uint32_t word, int backward, const DevLevel* coarse, const void* psi,
                            int variant, int cpb_override, bool snap) {
  if (L.mcur == nullptr || L.dim != 2 || theta_in == theta_out) return hipErrorInvalidValue;
  if (coarse != nullptr && psi == nullptr) return hipErrorInvalidValue;
  if (!L.fp32 && L.bm_table == nullptr) return hipErrorInvalidValue;
  // the kernel takes a shared right-hand side on the 5-point level and one
  // per chain on 9-point levels
  if (lv.cross ? fcs != 0 : (f == nullptr || fcs == 0)) return hipErrorInvalidValue;
  const int n = lv.g.n;
  const bool big = variant == 1;
  const bool dma = variant == 2 && lv.cross;  // LDS DMA tiles (5-point levels)
  if (snap && (lv.bsnap == nullptr || lv.bt_ptr[big ? 2 : 1] == nullptr)) return hipErrorInvalidValue;
  const BSnap bs = make_snap(lv, big ? 2 : 1, snap);
  const int tys = lv.cross ? (big ? 26 : 12) : (big ? 22 : 8);
  const int nt = big ? 512 : 256;
  const int tiles_x = (n + 63) / 64, tiles_y = (n + tys - 1) / tys;
  const int64_t tiles = int64_t(tiles_x) * tiles_y;
  int cpb = cpb_override > 0 ? cpb_override : chains_per_block(L.nchains, tiles);
  if (cpb > L.nchains) cpb = L.nchains;
  dim3 grid(unsigned(tiles), unsigned((L.nchains + cpb - 1) / cpb));
  const bool pro = coarse != nullptr;
  const bool userp = pro && lv.wP != nullptr;
  const Geom gc = pro ? coarse->g : Geom{};
#define MGMC_SEG_T(T, NP, PR, UP, TYS, NT, DM)                                                       \
  k_sweep2d_seg<T, NP, PR, UP, TYS, NT, 1, DM><<<grid, NT, 0, L.stream>>>(                          \
      (const T*)lv.coef, (const T*)lv.invd, (const T*)lv.isqd, (const T*)theta_in, (T*)theta_out,     \
      zero_in, (const T*)f, fcs, lv.g, (const T*)psi, gc, userp ? lv.wP : nullptr, backward, word,     \
      L.mcur, L.seed, L.chain0, tiles_x, cpb, L.nchains, L.bm_table, bs)
#define MGMC_SEG_NP(T, NP, TYS, NT, DM)                             \
  do {                                                              \
    if (!pro) MGMC_SEG_T(T, NP, false, false, TYS, NT, DM);         \
    else if (!userp) MGMC_SEG_T(T, NP, true, false, TYS, NT, DM);   \
    else MGMC_SEG_T(T, NP, true, true, TYS, NT, DM);                \
  } while (0)
#define MGMC_SEG_V(T)                                                          \
  do {                                                                         \
    if (lv.cross) {                                                            \
      if (big) MGMC_SEG_NP(T, 2, 26, 512, false);                              \
      else if (dma) MGMC_SEG_NP(T, 2, 12, 256, true);                          \
      else MGMC_SEG_NP(T, 2, 12, 256, false);                                  \
    } else {                                                                   \
      if (big) MGMC_SEG_NP(T, 4, 22, 512, false); else MGMC_SEG_NP(T, 4, 8, 256, false); \
    }                                                                          \
  } while (0)
  (void)tys;
  (void)nt;
  if (L.fp32) MGMC_SEG_V(float); else MGMC_SEG_V(double);
#undef MGMC_SEG_V
#undef MGMC_SEG_NP
#undef MGMC_SEG_T
  return hipGetLastError();
}

hipError_t launch_restrict_tiled(const Launch& L, const DevLevel& fine, const void* theta,
                                 const DevLevel& coarse, const void* f, int64_t fcs,
                                 const LowRankRhs& lr) {
  if (L.dim != 2) return hipErrorInvalidValue;
  constexpr int CTX = 32, CTY = 8;
  const int nc = coarse.g.n;
  const int tiles_x = (nc + CTX - 1) / CTX, tiles_y = (nc + CTY - 1) / CTY;
  const int64_t tiles = int64_t(tiles_x) * tiles_y;
  // as many chains per block as keep >= 1024 blocks (the operator is read
  // from memory once per chain group)
  int cpb = L.nchains;
  while (cpb > 1 && tiles * ((L.nchains + cpb - 1) / cpb) < 1024) cpb = (cpb + 1) / 2;
  dim3 grid(unsigned(tiles), unsigned((L.nchains + cpb - 1) / cpb));
  const bool userp = fine.wP != nullptr;
#define MGMC_RESTRICT_T(T, CR, UP, NT)                                                          \
  k_restrict2d_reg<T, CR, UP, CTY, NT><<<grid, NT, 0, L.stream>>>(                               \
      (const T*)fine.coef, (const T*)theta, (const T*)f, fcs, fine.g, (T*)coarse.f, coarse.g,       \
      fine.wP, tiles_x, cpb, L.nchains, lr)
#define MGMC_RESTRICT_P(T)                                                                      \
  do {                                                                                          \
    if (fine.cross) {                                                                           \
      if (userp) MGMC_RESTRICT_T(T, true, true, 256); else MGMC_RESTRICT_T(T, true, false, 256);  \
    } else {                                                                                    \
      if (userp) MGMC_RESTRICT_T(T, false, true, 512); else MGMC_RESTRICT_T(T, false, false, 512); \
    }                                                                                           \
  } while (0)
  if (L.fp32) MGMC_RESTRICT_P(float); else MGMC_RESTRICT_P(double);
#undef MGMC_RESTRICT_P
#undef MGMC_RESTRICT_T
  return hipGetLastError();
}

}  // namespace mgmc
