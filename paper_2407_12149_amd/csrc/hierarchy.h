// Host-side construction of the MGMC level hierarchy on structured grids.
//
// Every operator is a 3^dim-point stencil per site (entry t of site i couples
// i to i + delta(t), t = sum_k (delta_k + 1) 3^k, so ascending t is ascending
// neighbour index).  The finest operator has only the centre and the 2*dim
// axis entries; Galerkin coarse operators fill all 3^dim entries.
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
  double h = 0, scale = 0;
  std::vector<HostLevel> lv;   // lv[0] coarsest .. lv[L] finest
  int beta = 0;
  std::vector<double> gamma;
  // Coarsest exact sampler: theta_0 = K f_0 + U^{-1} z with At_0 = U^T U and
  // K = At_0^{-1}; both row-major.
  std::vector<double> K, Uinv;
};

// Forward colour order (colour id c = sum_k (i_k mod 2) 2^k): even parity sum
// first, then odd; backward sweeps use the reverse.
int forward_colour(int dim, int q);

// Returns MGMC_OK or an error code with a message in err.
mgmc_status build_hierarchy(const mgmc_problem& p, const mgmc_obs* obs, HostHierarchy& H,
                            std::string& err);

// f_L = B_L Gamma^{-1} y on the finest level (unpadded lexicographic).
std::vector<double> posterior_rhs(const HostHierarchy& H, const double* y);

}  // namespace mgmc
