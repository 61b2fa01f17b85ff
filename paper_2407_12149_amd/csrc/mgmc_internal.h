// Device-side data of the MGMC library and the kernel launchers.
//
// Layout of every level vector (state theta, right-hand side f, stencil
// arrays): padded lexicographic with a zero ghost ring, x fastest.  Node
// (i1, i2, i3), 0 <= i_k <= n+1, sits at (i1 + 3) + px (i2 + py i3) with
// px = round_up(n + 5, 4) and py = n + 2, so that interior node i1 = 4q + 1
// starts a 32-byte aligned group of four.  Chains are stored one padded field
// after another (chain-major).  Ghost entries are zero and never written.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace mgmc {

struct Geom {
  int n = 0;       // interior nodes per dimension
  int px = 0;      // x pitch
  int py = 0;      // rows per plane (n + 2)
  int64_t Np = 0;  // padded entries per field
  int64_t o0 = 0;  // offset of row 0 (px with a two-node halo, else 0)
};

// halo 1: the layout above.  halo 2 (2D levels with 5 x 5 stencils): rows
// -1 .. n+2 and x positions from i1 = -3, so node (i1, i2) sits at
// o0 + (i1 + 3) + px i2 with o0 = px, px = round_up(n + 6, 4), py = n + 4;
// every reach of two nodes from an interior node stays inside the field.
Geom make_geom(int dim, int n, int halo = 1);

struct DevLevel {
  Geom g;
  int64_t N = 0;                 // n^dim interior sites
  bool cross = false;            // stencil has only centre + axis entries
  void* coef = nullptr;          // [S][Np] stencil entries, precision T
  void* invd = nullptr;          // [Np] 1 / A_ii
  void* isqd = nullptr;          // [Np] 1 / sqrt(A_ii)
  double* wP = nullptr;          // [S][Np of level l-1] user prolongation into this level
  void* buf[2] = {nullptr, nullptr};  // two [nchains][Np] state buffers: tiled sweeps read
                                      // one and write the other (halos stay pre-sweep)
  void* f = nullptr;             // [nchains][Np] (levels below the finest)
  // observations B_l: columns (for B^T theta) and rows (for coarse rhs)
  int64_t* bptr = nullptr;       // [beta + 1]
  int64_t bnnz = 0;              // entries of B_l
  int32_t* bidx = nullptr;       // padded site of each weight
  double* bval = nullptr;
  int32_t nbrows = 0;
  int32_t* brow = nullptr;       // padded site of each row
  int64_t* brptr = nullptr;      // [nbrows + 1]
  int32_t* brcol = nullptr;      // observation index
  double* brval = nullptr;
  int32_t* brow_of = nullptr;    // [Np]: row of B_l at a padded site, -1 if none
  // low-rank smoother for forward (0) / backward (1) sweeps
  int32_t nsupp[2] = {0, 0};
  int32_t* supp[2] = {nullptr, nullptr};   // padded sites
  double* GT[2] = {nullptr, nullptr};      // [beta][nsupp], G = C S^{-1}
  double* SinvT = nullptr;                 // [beta][beta], S^{-1} of the forward sweep, transposed
  // B^T theta without a separate pass over theta (2D one-launch sweeps): the
  // sweep kernels write B's weight times the swept value at each of B's
  // sites into bsnap.  Its layout gives every column of B the same number
  // bkp (8, 9, 12, 16 or 32) of slots: [nchains][beta][bkp], column j's entries
  // in the order of bidx, then zeros, which stay zero (bpval holds the
  // weights in the same slots).  bt_ptr / bt_ent list the slots whose site
  // lies in each 64 x TY tile, for the tile heights of the three 2D sweep
  // forms (kSnapTY).
  int bkp = 0;
  int64_t bslots = 0;                                // beta * bkp
  double* bpval = nullptr;                           // [beta][bkp] weights, zero padded
  int32_t* bpidx = nullptr;                          // [beta][bkp] padded sites (0 on padding)
  int32_t* bt_ptr[3] = {nullptr, nullptr, nullptr};  // [tiles + 1]
  int32_t* bt_ent[3] = {nullptr, nullptr, nullptr};  // [bnnz] slots
  double* bsnap = nullptr;
};

// Tile heights of the 2D sweep forms, as indexed by DevLevel::bt_ptr: the
// LDS-tiled sweep, and the segment sweep with 256 and 512 threads, for
// 5-point (cross) and 9-point levels.
constexpr int kSnapTY[2][3] = {{32, 8, 22}, {32, 12, 26}};

// Kernel argument: where a 2D sweep writes the snapshot of B's sites.
struct BSnap {
  const int32_t* ptr = nullptr;  // bt_ptr of the sweep's tile height
  const int32_t* ent = nullptr;  // slots
  const int32_t* idx = nullptr;  // bpidx
  const double* w = nullptr;     // bpval
  double* snap = nullptr;        // null: no snapshot
  int64_t nnz = 0;               // slots per chain (beta * bkp)
};

// The low-rank part of the restricted residual, B_{l-1} v with
// v = Gamma^{-1} B_l^T theta (per chain), added by the restriction kernels.
struct LowRankRhs {
  const int32_t* row_of = nullptr;  // coarse level: row of B_{l-1} at a padded site, or -1
  const int64_t* ptr = nullptr;
  const int32_t* col = nullptr;
  const double* val = nullptr;
  const double* v = nullptr;        // [nchains][beta]
  int beta = 0;
};

// Arguments of the one-launch bottom of the V-cycle (kernels_coarse.hip):
// levels 0..lm of a 2D hierarchy, all Galerkin 9-point.
constexpr int kMaxCoarseLevels = 6;
struct CoarseLevel {
  Geom g;
  const void* coef = nullptr;  // [9][Np], state precision
  const void* invd = nullptr;
  const void* isqd = nullptr;
  const int64_t* bptr = nullptr;  // B_l by columns (padded sites)
  const int32_t* bidx = nullptr;
  const double* bval = nullptr;
  int32_t nsupp[2] = {0, 0};
  const int32_t* supp[2] = {nullptr, nullptr};
  const double* GT[2] = {nullptr, nullptr};
  const double* SinvT = nullptr;
  const int32_t* brow_of = nullptr;  // B_l by rows (restriction into this level)
  const int64_t* brptr = nullptr;
  const int32_t* brcol = nullptr;
  const double* brval = nullptr;
};
struct CoarseCommon {
  int beta = 0, nu1 = 1, nu2 = 1;
  const double* gisq = nullptr;
  const double* gam = nullptr;
  const double* K = nullptr;
  const double* Uinv = nullptr;
  const int64_t* mcur = nullptr;
  uint32_t seed = 0, chain0 = 0;
};
struct CoarseArgs {
  int lm = 0;
  CoarseLevel L[kMaxCoarseLevels];
  CoarseCommon C;
  const void* f_top = nullptr;  // [nchains][Np of level lm]: right-hand side of level lm
  void* theta_top = nullptr;    // [nchains][Np of level lm]: its state after the post-sweeps
};
// LDS bytes of the launch, the one-time attribute set-up (above 64 KiB) and
// the launch itself (one workgroup of 512 threads per chain).
size_t coarse_vcycle_lds(const CoarseArgs& a, bool fp32, int64_t max_bnnz);
hipError_t coarse_vcycle_prepare(bool fp32, size_t lds_bytes);
hipError_t launch_coarse_vcycle(const struct Launch& L, const CoarseArgs& a, size_t lds_bytes);

struct Launch {
  hipStream_t stream = nullptr;
  int dim = 2;
  int fp32 = 0;
  int nchains = 1;
  uint32_t seed = 0;
  uint32_t chain0 = 0;
  const int64_t* mcur = nullptr;  // device: current sample index
  int lowrank_mfma = 0;           // low-rank G t product on the matrix cores
  const double* bm_table = nullptr;  // device: Box-Muller table (device_rng.h), kBmTable doubles
  int cpb_force = 0;  // > 0: chains per thread of the per-site kernels (3D contexts), else by size
  double omega = 1.0;  // SOR relaxation of the per-colour sweeps (others need 1)
  int march3d = 0;     // z-marching 3D sweep form: 1 tiles of 24 rows, 2 of 8 rows
  int restrict3d = 1;  // 3D 7-point levels: residual and restriction in one launch
};

// Chains per thread (or block) for kernels that keep a site's stencil in
// registers across chains: up to 16, doubled while at least ~2048 blocks
// would remain; force > 0 sets it (capped at 16 and at nchains).
inline int chain_group(int64_t blocks, int nchains, int force = 0) {
  if (force > 0) return std::min(std::min(force, 16), nchains);
  int cpb = 1;
  while (cpb < 16 && cpb < nchains && blocks * ((nchains + 2 * cpb - 1) / (2 * cpb)) >= 2048) cpb *= 2;
  return cpb;
}

// Host: fill the Box-Muller table of gauss_pair_tab (device_rng.h).
constexpr int kBmTable = 770;
void fill_bm_table(double* t);

// Noise counter word 1: visit << 16 | level << 8 | sweep << 4 | colour, the
// visit counting the calls of a level within one update (W-cycles).
__host__ __device__ inline uint32_t noise_word(int level, int sigma, int visit = 0) {
  return (uint32_t(visit) << 16) | (uint32_t(level) << 8) | (uint32_t(sigma) << 4);
}

// One colour pass, in place on theta.
hipError_t launch_sweep_colour(const Launch& L, const DevLevel& lv, void* theta, const void* f,
                               int64_t fcs, uint32_t word, int colour);
// Parity pass (0: even parity sum first in forward order, 1: odd) of a 3D
// sweep on a 7-point level, in place.
hipError_t launch_sweep_parity3d(const Launch& L, const DevLevel& lv, void* theta, const void* f,
                                 int64_t fcs, uint32_t word, int parity);
// LDS-tiled 2D sweep (all colour passes in one launch) from theta_in into
// theta_out (distinct buffers).  zero_in: the input state is zero (not read).
// coarse != nullptr adds the prolongation P psi of the coarse state psi while
// loading.
hipError_t launch_sweep_tiled(const Launch& L, const DevLevel& lv, const void* theta_in,
                              void* theta_out, int zero_in, const void* f, int64_t fcs,
                              uint32_t word, int backward, const DevLevel* coarse, const void* psi,
                              bool snap = false);
// Segment form of the tiled sweep (stencil held in registers across passes
// and chains).  variant 0: 256 threads per block, 1: 512, 2: 256 with the
// state tiles copied into LDS by DMA, double-buffered across chains
// (5-point levels; 9-point levels take variant 0); cpb_override > 0 fixes
// the chains per block.
hipError_t launch_sweep_seg(const Launch& L, const DevLevel& lv, const void* theta_in,
                            void* theta_out, int zero_in, const void* f, int64_t fcs,
                            uint32_t word, int backward, const DevLevel* coarse, const void* psi,
                            int variant, int cpb_override, bool snap = false);
// Restriction f_{l-1} = P^T (f_l - A_l theta) - B_{l-1} v (the last term
// from lr when lr.row_of is set).
hipError_t launch_restrict_tiled(const Launch& L, const DevLevel& fine, const void* theta,
                                 const DevLevel& coarse, const void* f, int64_t fcs,
                                 const LowRankRhs& lr);
hipError_t launch_restrict(const Launch& L, const DevLevel& fine, const void* theta,
                           const DevLevel& coarse, const void* f, int64_t fcs,
                           const LowRankRhs& lr);
// Residual into scratch (a second state buffer of the fine level), then
// restriction of the residual: for 3D, where a coarse node's support is large.
hipError_t launch_restrict_2stage(const Launch& L, const DevLevel& fine, const void* theta,
                                  void* scratch, const DevLevel& coarse, const void* f,
                                  int64_t fcs, const LowRankRhs& lr);
// Residual and restriction of a 3D 7-point level (multilinear weights) in one
// launch over LDS tiles; used by launch_restrict_2stage when L.restrict3d.
hipError_t launch_restrict3d_lds(const Launch& L, const DevLevel& fine, const void* theta,
                                 const DevLevel& coarse, const void* f, int64_t fcs,
                                 const LowRankRhs& lr);
hipError_t launch_prolong(const Launch& L, const DevLevel& fine, void* theta,
                          const DevLevel& coarse, const void* psi);
hipError_t launch_coarsest(const Launch& L, const DevLevel& lv0, const void* f0, int64_t fcs,
                           void* theta0, const double* K, const double* Uinv, uint32_t word = 0);
// One-launch sweep of a 3D 7-point level (both parity passes), marching in
// z over LDS x-y tiles, from theta_in into theta_out (distinct buffers).
hipError_t launch_sweep3d_march(const Launch& L, const DevLevel& lv, const void* theta_in,
                                void* theta_out, const void* f, uint32_t word, int backward);
// Levels with 5 x 5 stencils (2D, nine colours (i_1 mod 3) + 3 (i_2 mod 3)):
// one colour pass in place, and the residual into scratch followed by the
// restriction P^T r (minus B_{l-1} v).
hipError_t launch_sweep_wide(const Launch& L, const DevLevel& lv, void* theta, const void* f,
                             int64_t fcs, uint32_t word, int colour);
hipError_t launch_restrict_wide(const Launch& L, const DevLevel& fine, const void* theta,
                                void* scratch, const DevLevel& coarse, const void* f, int64_t fcs,
                                const LowRankRhs& lr);
hipError_t launch_restrict_residual(const Launch& L, const DevLevel& fine, const void* r,
                                    const DevLevel& coarse, const LowRankRhs& lr);
// Exact single-level sample theta = mu + U^{-1} z with the banded factor
// U (N rows of band + 1 entries, FP64): x ([nchains][N] FP64 scratch) takes
// the normals z (tag 2, counter word `word`), the back substitution runs in
// place, and theta (padded, state precision) receives mu + x; mu may be null
// (f = 0).
hipError_t launch_band_sample(const Launch& L, const DevLevel& lv, const double* U, int64_t band,
                              const double* mu, double* x, void* theta, uint32_t word);
// Low-rank correction after a sweep in direction dir (Alg. 3):
// theta -= G (B^T theta - Gamma xi) with xi = Gamma^{-1/2} zeta; t receives
// B^T theta - Gamma xi per chain ([nchains][beta] scratch).  v_out != nullptr
// (forward sweeps) also receives v = Gamma^{-1} B^T theta' = xi + S^{-1} t.
hipError_t launch_lowrank(const Launch& L, const DevLevel& lv, void* theta, int dir, uint32_t word,
                          int beta, const double* gisq, const double* gam, double* t,
                          double* v_out);
// The same correction for a level whose sweep just wrote its snapshot of B's
// sites (lv.bsnap): one launch forms t = B^T theta - Gamma xi from the
// snapshot in every block and applies theta -= G t on the matrix cores
// (beta <= 128); with v_out it also writes v = xi + S^{-1} t.
hipError_t launch_lowrank_fused(const Launch& L, const DevLevel& lv, void* theta, int dir,
                                uint32_t word, int beta, const double* gisq, const double* gam,
                                double* v_out);
hipError_t launch_fill_zero(const Launch& L, void* p, int64_t count);
// q = F^T theta per chain into qoi[m - m0][chain], then m += 1 (the last
// launches of an update).  partial: nb * nchains doubles.
constexpr int kQoiChains = 8;  // chains per block of the partial sums
hipError_t launch_qoi(const Launch& L, const DevLevel& fine, const void* theta, const double* F,
                      double* partial, int nb, double* qoi, int64_t m0);
hipError_t launch_unpack(const Launch& L, const DevLevel& lv, const void* user, void* theta);
hipError_t launch_pack(const Launch& L, const DevLevel& lv, const void* theta, void* user);
hipError_t launch_unpack_rhs(const Launch& L, const DevLevel& lv, const double* user, void* f);
// dst[c] = src (padded, state precision) for every chain, or 0 where src is null.
hipError_t launch_broadcast(const Launch& L, const DevLevel& lv, const void* src, void* dst);
hipError_t launch_set_m(hipStream_t s, int64_t* mcur, int64_t value);
hipError_t launch_advance_m(hipStream_t s, int64_t* mcur);

}  // namespace mgmc
