// Host-side construction of the MGMC level hierarchy on structured grids.
//
// Every operator is a (2R+1)^dim-point stencil per site (entry t of site i
// couples i to i + delta(t), t = sum_k (delta_k + R) (2R+1)^k, so ascending t
// is ascending neighbour index), R = 1 except for the 13-point squared shifted
// Laplace (R = 2).  The finite-difference fine operator has only the centre
// and the 2*dim axis entries; Galerkin coarse operators fill the stencil.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "mgmc.h"

namespace mgmc {

struct HostLevel {
  int n = 0;                  // interior nodes per dimension
  int64_t N = 0;              // n^dim sites
  std::vector<double> st;     // stencil, st[t * N + i]
  // Weights of the prolongation from the next coarser level into this one,
  // per coarse node: wP[J * S + t] (only for user weights on the finest
  // transfer; empty means multilinear).
  std::vector<double> wP;
  // Observation matrix B_l by columns: sorted (site, weight) lists.
  std::vector<std::vector<std::pair<int64_t, double>>> Bcol;
  // Low-rank smoother for forward (0) and backward (1) sweeps (Alg. 3):
  // rows where C = M^{-1} B is non-zero, C and G = C S^{-1} on those rows
  // (row-major nsupp x beta), S - Gamma = B^T C and S^{-1} (beta x beta,
  // row-major).
  std::vector<int64_t> supp[2];
  std::vector<double> C[2], G[2], SmG[2], Sinv[2];
};

struct HostHierarchy {
  int dim = 2, L = 0, S = 9, ncolours = 4;
  int R = 1;           // stencil radius; colour classes per axis q = R + 1
  int op = 0;          // MGMC_OP_*
  double omega = 1.0;  // SOR relaxation of the Gibbs sweeps
  bool level0_lowrank = false;  // level 0 is smoothed (Alg. 5 or the Gibbs sampler)
  double h = 0, scale = 0;
  std::vector<HostLevel> lv;   // lv[0] coarsest .. lv[L] finest
  int beta = 0;
  std::vector<double> gamma;
  // Coarsest exact sampler: theta_0 = K f_0 + U^{-1} z with At_0 = U^T U and
  // K = At_0^{-1}; both row-major (empty when level 0 is smoothed or sampled
  // by the banded factor below).
  std::vector<double> K, Uinv;
  // Exact sampler of a single level by a banded Cholesky factor At = U^T U in
  // lexicographic order: row i of U holds U(i, i .. i + band) at
  // Uband[i * (band + 1) + (j - i)].
  int64_t band = 0;
  std::vector<double> Uband;
};

// Forward colour order.  With two classes per axis (colour id c = sum_k
// (i_k mod 2) 2^k): even parity sum first, then odd; with three classes
// (2D, c = (i_1 mod 3) + 3 (i_2 mod 3)): ascending.  Backward sweeps use the
// reverse.
int forward_colour(int dim, int nclass, int q);

// Banded Cholesky factor of the finest At (single-level exact sampler).
mgmc_status band_cholesky(HostHierarchy& H, std::string& err);
// mu = At^{-1} f with the banded factor (forward then backward substitution).
std::vector<double> band_solve(const HostHierarchy& H, const double* f);

// Returns MGMC_OK or an error code with a message in err.
mgmc_status build_hierarchy(const mgmc_problem& p, const mgmc_obs* obs, HostHierarchy& H,
                            std::string& err);

// f_L = B_L Gamma^{-1} y on the finest level (unpadded lexicographic).
std::vector<double> posterior_rhs(const HostHierarchy& H, const double* y);

}  // namespace mgmc
