// Structured construction of the MGMC hierarchy (host, FP64).
//
//  * fine operator (paper Sec. 5.1.1): s (kappa^2 I - div(a grad)) by finite
//    differences with face coefficients and zero Dirichlet data, bilinear
//    finite elements for -Laplace + kappa^2, or the 13-point squared shifted
//    Laplace with clamped boundaries;
//  * prolongation: column J of P carries w_J(delta) at fine node 2J + delta,
//    multilinear by default (Sec. 3.1, Sec. 5.1.3 "Samplers");
//  * Galerkin coarse operators A_{l-1} = P^T A_l P and B_{l-1} = P^T B_l
//    (eq. A_ell_1_B_ell_1), assembled stencil-wise;
//  * low-rank smoother data C = M^{-1} B, S = Gamma + B^T C, G = C S^{-1}
//    (Alg. 3, M = D / omega + L in colour order);
//  * the coarsest exact sampler from the Cholesky factor At_0 = U^T U
//    (Sec. 3.5 and the Cholesky sampler of Sec. 5.1.3).
#include "hierarchy.h"

#include <algorithm>
#include <cmath>
#include <map>
#include <thread>

namespace mgmc {

namespace {

constexpr int kFwd2[4] = {0, 3, 1, 2};
constexpr int kFwd3[8] = {0, 3, 5, 6, 1, 2, 4, 7};

struct Geo {
  int dim, n;
  int64_t N;
  void coords(int64_t lin, int* i) const {
    for (int k = 0; k < dim; ++k) {
      i[k] = 1 + int(lin % n);
      lin /= n;
    }
  }
  int64_t lin(const int* i) const {
    int64_t v = 0;
    for (int k = dim - 1; k >= 0; --k) v = v * n + (i[k] - 1);
    return v;
  }
};

// Stencil entry of offset d in a stencil of radius R.
inline int stencil_index(int dim, int R, const int* d) {
  int t = 0, m = 1;
  for (int k = 0; k < dim; ++k) {
    t += (d[k] + R) * m;
    m *= 2 * R + 1;
  }
  return t;
}

inline void stencil_delta(int dim, int R, int t, int* d) {
  for (int k = 0; k < dim; ++k) {
    d[k] = t % (2 * R + 1) - R;
    t /= 2 * R + 1;
  }
}

// Multilinear weight of prolongation offset delta (t = index of delta in the
// 3^dim box), or the user's weight of coarse node J.
inline double pweight(const HostLevel& fine, int dim, int64_t J, int t) {
  const int SP = dim == 2 ? 9 : 27;
  if (!fine.wP.empty()) return fine.wP[size_t(J) * SP + t];
  int d[3];
  stencil_delta(dim, 1, t, d);
  double w = 1.0;
  for (int k = 0; k < dim; ++k)
    if (d[k] != 0) w *= 0.5;
  return w;
}

template <class F>
void parallel_for(int64_t count, F&& body) {
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (count < 4096 || nt == 1) {
    body(int64_t(0), count);
    return;
  }
  std::vector<std::thread> th;
  int64_t chunk = (count + nt - 1) / nt;
  for (unsigned w = 0; w < nt; ++w) {
    int64_t b = int64_t(w) * chunk, e = std::min(count, b + chunk);
    if (b < e) th.emplace_back([&body, b, e] { body(b, e); });
  }
  for (auto& t : th) t.join();
}

void fine_operator(const mgmc_problem& p, HostHierarchy& H) {
  HostLevel& f = H.lv[H.L];
  const int dim = p.dim, n = p.n, S = H.S;
  Geo g{dim, n, f.N};
  f.st.assign(size_t(S) * f.N, 0.0);
  const double s = H.scale, ih2 = 1.0 / (H.h * H.h);
  int64_t per = n + 1;
  for (int k = 1; k < dim; ++k) per *= n;
  auto face = [&](int k, const int* i, int fk) -> double {
    if (!p.face_coef) return 1.0;
    int64_t idx = 0, mult = 1;
    for (int j = 0; j < dim; ++j) {
      idx += int64_t(j == k ? fk : i[j] - 1) * mult;
      mult *= (j == k) ? n + 1 : n;
    }
    return p.face_coef[k * per + idx];
  };
  const int centre = (S - 1) / 2;
  parallel_for(f.N, [&](int64_t b, int64_t e) {
    int i[3], d[3];
    for (int64_t lin = b; lin < e; ++lin) {
      g.coords(lin, i);
      double faces = 0.0;
      for (int k = 0; k < dim; ++k) {
        double ap = face(k, i, i[k]), am = face(k, i, i[k] - 1);
        faces += ap + am;
        for (int j = 0; j < dim; ++j) d[j] = 0;
        if (i[k] < n) {
          d[k] = 1;
          f.st[size_t(stencil_index(dim, 1, d)) * f.N + lin] = -s * ih2 * ap;
        }
        if (i[k] > 1) {
          d[k] = -1;
          f.st[size_t(stencil_index(dim, 1, d)) * f.N + lin] = -s * ih2 * am;
        }
      }
      f.st[size_t(centre) * f.N + lin] = s * p.kappa2 + s * ih2 * faces;
    }
  });
}

// Bilinear (Q1) finite elements for -Laplace + kappa^2 on the uniform 2D grid
// (Sec. 5.1.1): each site's 9-point row is the sum, over the four cells
// around it, of the element stiffness (1/6)[4 -1 -2 -1; ...] and kappa^2 times
// the element mass (h^2/36)[4 2 1 2; ...] between the site's corner and the
// neighbour's corner of that cell, scaled by s / h^2.  Couplings to boundary
// nodes are dropped (u = 0 there).
void fem_q1_operator(const mgmc_problem& p, HostHierarchy& H) {
  HostLevel& f = H.lv[H.L];
  const int n = p.n;
  f.st.assign(size_t(H.S) * f.N, 0.0);
  const double h = H.h, sc = H.scale / (h * h);
  // element matrices, corners counter-clockwise from the lower left
  const double KE[4][4] = {{4, -1, -2, -1}, {-1, 4, -1, -2}, {-2, -1, 4, -1}, {-1, -2, -1, 4}};
  const double ME[4][4] = {{4, 2, 1, 2}, {2, 4, 2, 1}, {1, 2, 4, 2}, {2, 1, 2, 4}};
  const int CX[4] = {0, 1, 1, 0}, CY[4] = {0, 0, 1, 1};
  Geo g{2, n, f.N};
  parallel_for(f.N, [&](int64_t b, int64_t e) {
    int i[2], d[2];
    for (int64_t lin = b; lin < e; ++lin) {
      g.coords(lin, i);
      for (int a = 0; a < 4; ++a) {  // the site is corner a of the cell
        const int cx = i[0] - CX[a], cy = i[1] - CY[a];
        for (int bb = 0; bb < 4; ++bb) {
          const int j0 = cx + CX[bb], j1 = cy + CY[bb];
          if (j0 < 1 || j0 > n || j1 < 1 || j1 > n) continue;
          d[0] = j0 - i[0];
          d[1] = j1 - i[1];
          const double v = KE[a][bb] / 6.0 + p.kappa2 * (h * h) * ME[a][bb] / 36.0;
          f.st[size_t(stencil_index(2, 1, d)) * f.N + lin] += sc * v;
        }
      }
    }
  });
}

// Squared shifted Laplace (Sec. 5.1.1), 2D:
// s [h^-4 B13 + 2 kappa^2 h^-2 L5 + kappa^4 I] with the 13-point biharmonic
// difference B13 (20 at the centre, -8 at the axis neighbours, 2 at the
// diagonal ones, 1 two steps along an axis) and the 5-point -Laplace L5.
// Clamped boundary: boundary nodes are 0, and a reach to the ghost node one
// step outside the boundary lands on the interior node it mirrors.
void ssl13_operator(const mgmc_problem& p, HostHierarchy& H) {
  HostLevel& f = H.lv[H.L];
  const int n = p.n;
  f.st.assign(size_t(H.S) * f.N, 0.0);
  const double s = H.scale, ih2 = 1.0 / (H.h * H.h), ih4 = ih2 * ih2, k2 = p.kappa2;
  const int OFF[13][2] = {{0, 0},  {1, 0},   {-1, 0}, {0, 1}, {0, -1}, {1, 1}, {1, -1},
                          {-1, 1}, {-1, -1}, {2, 0},  {-2, 0}, {0, 2}, {0, -2}};
  const double WB[13] = {20, -8, -8, -8, -8, 2, 2, 2, 2, 1, 1, 1, 1};
  Geo g{2, n, f.N};
  parallel_for(f.N, [&](int64_t b, int64_t e) {
    int i[2], j[2], d[2];
    for (int64_t lin = b; lin < e; ++lin) {
      g.coords(lin, i);
      for (int t = 0; t < 13; ++t) {
        bool skip = false;
        for (int k = 0; k < 2; ++k) {
          j[k] = i[k] + OFF[t][k];
          if (j[k] == 0 || j[k] == n + 1) skip = true;
          if (j[k] == -1) j[k] = 1;
          if (j[k] == n + 2) j[k] = n;
          d[k] = j[k] - i[k];
        }
        if (!skip) f.st[size_t(stencil_index(2, 2, d)) * f.N + lin] += s * ih4 * WB[t];
      }
      for (int t = 0; t < 5; ++t) {
        bool skip = false;
        for (int k = 0; k < 2; ++k) {
          j[k] = i[k] + OFF[t][k];
          if (j[k] < 1 || j[k] > n) skip = true;
          d[k] = OFF[t][k];
        }
        if (!skip)
          f.st[size_t(stencil_index(2, 2, d)) * f.N + lin] += s * 2.0 * k2 * ih2 * (t == 0 ? 4.0 : -1.0);
      }
      d[0] = d[1] = 0;
      f.st[size_t(stencil_index(2, 2, d)) * f.N + lin] += s * k2 * k2;
    }
  });
}

// A_c = P^T A_f P, stencil by stencil: for coarse node J, every fine node
// i = 2J + d1 in the support of column J couples through A_f to fine j, and j
// lies in the support of the columns K covering it.
void galerkin(const HostHierarchy& H, int lf, HostLevel& c) {
  const HostLevel& f = H.lv[lf];
  const int dim = H.dim, S = H.S, R = H.R, nf = f.n, nc = c.n;
  const int SP = dim == 2 ? 9 : 27;  // prolongation offsets {-1,0,1}^dim
  Geo gf{dim, nf, f.N}, gc{dim, nc, c.N};
  c.st.assign(size_t(S) * c.N, 0.0);
  parallel_for(c.N, [&](int64_t b, int64_t e) {
    int J[3], d1[3], d2[3], i[3], j[3], K[3], opts[3][2], dl[3][2], nopt[3];
    for (int64_t Jl = b; Jl < e; ++Jl) {
      gc.coords(Jl, J);
      for (int t1 = 0; t1 < SP; ++t1) {
        stencil_delta(dim, 1, t1, d1);
        for (int k = 0; k < dim; ++k) i[k] = 2 * J[k] + d1[k];
        const double w1 = pweight(f, dim, Jl, t1);
        if (w1 == 0.0) continue;
        const int64_t il = gf.lin(i);
        for (int t2 = 0; t2 < S; ++t2) {
          const double a = f.st[size_t(t2) * f.N + il];
          if (a == 0.0) continue;
          stencil_delta(dim, R, t2, d2);
          bool inside = true;
          for (int k = 0; k < dim; ++k) {
            j[k] = i[k] + d2[k];
            if (j[k] < 1 || j[k] > nf) inside = false;
          }
          if (!inside) continue;
          // coarse nodes K covering j, with j = 2K + delta
          for (int k = 0; k < dim; ++k) {
            nopt[k] = 0;
            if ((j[k] & 1) == 0) {
              opts[k][0] = j[k] / 2; dl[k][0] = 0; nopt[k] = 1;
            } else {
              int lo = (j[k] - 1) / 2, hi = (j[k] + 1) / 2;
              if (lo >= 1) { opts[k][nopt[k]] = lo; dl[k][nopt[k]] = 1; ++nopt[k]; }
              if (hi <= nc) { opts[k][nopt[k]] = hi; dl[k][nopt[k]] = -1; ++nopt[k]; }
            }
          }
          int total = 1;
          for (int k = 0; k < dim; ++k) total *= nopt[k];
          for (int comb = 0; comb < total; ++comb) {
            int r = comb, dd[3], dk[3];
            for (int k = 0; k < dim; ++k) {
              int o = r % nopt[k];
              r /= nopt[k];
              K[k] = opts[k][o];
              dd[k] = dl[k][o];
              dk[k] = K[k] - J[k];
            }
            const double w2 = pweight(f, dim, gc.lin(K), stencil_index(dim, 1, dd));
            c.st[size_t(stencil_index(dim, R, dk)) * c.N + Jl] += w1 * a * w2;
          }
        }
      }
    }
  });
}

// B_{l-1} = P^T B_l column by column.
void restrict_observations(const HostHierarchy& H, int lf, HostLevel& c) {
  const HostLevel& f = H.lv[lf];
  const int dim = H.dim, nc = c.n;
  Geo gf{dim, f.n, f.N}, gc{dim, nc, c.N};
  c.Bcol.assign(f.Bcol.size(), {});
  for (size_t col = 0; col < f.Bcol.size(); ++col) {
    std::map<int64_t, double> acc;
    int i[3], K[3], opts[3][2], dl[3][2], nopt[3];
    for (const auto& [il, b] : f.Bcol[col]) {
      gf.coords(il, i);
      for (int k = 0; k < dim; ++k) {
        nopt[k] = 0;
        if ((i[k] & 1) == 0) {
          opts[k][0] = i[k] / 2; dl[k][0] = 0; nopt[k] = 1;
        } else {
          int lo = (i[k] - 1) / 2, hi = (i[k] + 1) / 2;
          if (lo >= 1) { opts[k][nopt[k]] = lo; dl[k][nopt[k]] = 1; ++nopt[k]; }
          if (hi <= nc) { opts[k][nopt[k]] = hi; dl[k][nopt[k]] = -1; ++nopt[k]; }
        }
      }
      int total = 1;
      for (int k = 0; k < dim; ++k) total *= nopt[k];
      for (int comb = 0; comb < total; ++comb) {
        int r = comb, dd[3];
        for (int k = 0; k < dim; ++k) {
          int o = r % nopt[k];
          r /= nopt[k];
          K[k] = opts[k][o];
          dd[k] = dl[k][o];
        }
        const int64_t Kl = gc.lin(K);
        acc[Kl] += pweight(f, dim, Kl, stencil_index(dim, 1, dd)) * b;
      }
    }
    c.Bcol[col].assign(acc.begin(), acc.end());
  }
}

// LU with partial pivoting of a dense m x m matrix, then the inverse.
bool dense_inverse(std::vector<double> a, int m, std::vector<double>& inv) {
  std::vector<int> perm(m);
  for (int r = 0; r < m; ++r) perm[r] = r;
  for (int c = 0; c < m; ++c) {
    int piv = c;
    for (int r = c + 1; r < m; ++r)
      if (std::fabs(a[size_t(r) * m + c]) > std::fabs(a[size_t(piv) * m + c])) piv = r;
    if (a[size_t(piv) * m + c] == 0.0) return false;
    if (piv != c) {
      for (int t = 0; t < m; ++t) std::swap(a[size_t(c) * m + t], a[size_t(piv) * m + t]);
      std::swap(perm[c], perm[piv]);
    }
    const double d = a[size_t(c) * m + c];
    for (int r = c + 1; r < m; ++r) {
      const double l = a[size_t(r) * m + c] / d;
      a[size_t(r) * m + c] = l;
      for (int t = c + 1; t < m; ++t) a[size_t(r) * m + t] -= l * a[size_t(c) * m + t];
    }
  }
  inv.assign(size_t(m) * m, 0.0);
  std::vector<double> x(m);
  for (int e = 0; e < m; ++e) {
    for (int r = 0; r < m; ++r) x[r] = (perm[r] == e) ? 1.0 : 0.0;
    for (int r = 0; r < m; ++r)
      for (int t = 0; t < r; ++t) x[r] -= a[size_t(r) * m + t] * x[t];
    for (int r = m - 1; r >= 0; --r) {
      for (int t = r + 1; t < m; ++t) x[r] -= a[size_t(r) * m + t] * x[t];
      x[r] /= a[size_t(r) * m + r];
    }
    for (int r = 0; r < m; ++r) inv[size_t(r) * m + e] = x[r];
  }
  return true;
}

// C = M^{-1} B by substitution in sweep order, restricted to the bounding box
// of each column's support dilated by (ncolours - 1): a colour pass can only
// spread non-zeros by one stencil radius.
mgmc_status lowrank_level(HostHierarchy& H, int l, std::string& err) {
  HostLevel& lv = H.lv[l];
  const int dim = H.dim, S = H.S, n = lv.n, beta = H.beta, nq = H.ncolours, R = H.R;
  const int q = R + 1;
  const int centre = (S - 1) / 2;
  Geo g{dim, n, lv.N};
  for (int dir = 0; dir < 2; ++dir) {
    std::vector<std::vector<std::pair<int64_t, double>>> Ccol(beta);
    parallel_for(beta, [&](int64_t jb, int64_t je) {
      for (int64_t j = jb; j < je; ++j) {
        int lo[3], hi[3], ext[3], i[3], d[3];
        for (int k = 0; k < dim; ++k) { lo[k] = n + 1; hi[k] = 0; }
        for (const auto& [il, b] : lv.Bcol[j]) {
          g.coords(il, i);
          for (int k = 0; k < dim; ++k) { lo[k] = std::min(lo[k], i[k]); hi[k] = std::max(hi[k], i[k]); }
        }
        if (lv.Bcol[j].empty()) continue;
        int64_t vol = 1;
        for (int k = 0; k < dim; ++k) {
          lo[k] = std::max(1, lo[k] - (nq - 1) * R);
          hi[k] = std::min(n, hi[k] + (nq - 1) * R);
          ext[k] = hi[k] - lo[k] + 1;
          vol *= ext[k];
        }
        auto boxlin = [&](const int* c) {
          int64_t v = 0;
          for (int k = dim - 1; k >= 0; --k) v = v * ext[k] + (c[k] - lo[k]);
          return v;
        };
        std::vector<double> x(vol, 0.0), b(vol, 0.0);
        for (const auto& [il, bv] : lv.Bcol[j]) {
          g.coords(il, i);
          b[boxlin(i)] = bv;
        }
        for (int qq = 0; qq < nq; ++qq) {
          const int colour = forward_colour(dim, q, dir == 0 ? qq : nq - 1 - qq);
          for (int64_t v = 0; v < vol; ++v) {
            int64_t r = v;
            int c = 0, mult = 1;
            for (int k = 0; k < dim; ++k) {
              i[k] = lo[k] + int(r % ext[k]);
              r /= ext[k];
              c += (i[k] % q) * mult;
              mult *= q;
            }
            if (c != colour) continue;
            const int64_t il = g.lin(i);
            double s = b[v];
            for (int t = 0; t < S; ++t) {
              if (t == centre) continue;
              const double a = lv.st[size_t(t) * lv.N + il];
              if (a == 0.0) continue;
              stencil_delta(dim, R, t, d);
              int jn[3];
              bool in = true;
              for (int k = 0; k < dim; ++k) {
                jn[k] = i[k] + d[k];
                if (jn[k] < lo[k] || jn[k] > hi[k]) in = false;
              }
              if (in) s -= a * x[boxlin(jn)];
            }
            x[v] = (H.omega * s) / lv.st[size_t(centre) * lv.N + il];
          }
        }
        for (int64_t v = 0; v < vol; ++v) {
          if (x[v] == 0.0) continue;
          int64_t r = v;
          for (int k = 0; k < dim; ++k) {
            i[k] = lo[k] + int(r % ext[k]);
            r /= ext[k];
          }
          Ccol[j].push_back({g.lin(i), x[v]});
        }
        std::sort(Ccol[j].begin(), Ccol[j].end());
      }
    });
    std::vector<int64_t> rows;
    for (int j = 0; j < beta; ++j)
      for (const auto& e : Ccol[j]) rows.push_back(e.first);
    std::sort(rows.begin(), rows.end());
    rows.erase(std::unique(rows.begin(), rows.end()), rows.end());
    const int64_t ns = int64_t(rows.size());
    std::vector<double> Cs(size_t(ns) * beta, 0.0);
    auto where = [&](int64_t site) {
      auto it = std::lower_bound(rows.begin(), rows.end(), site);
      return (it != rows.end() && *it == site) ? int64_t(it - rows.begin()) : int64_t(-1);
    };
    for (int j = 0; j < beta; ++j)
      for (const auto& [site, v] : Ccol[j]) Cs[size_t(where(site)) * beta + j] = v;
    // S = Gamma + B^T C
    std::vector<double> Sm(size_t(beta) * beta, 0.0), SmG(size_t(beta) * beta, 0.0);
    for (int a = 0; a < beta; ++a)
      for (const auto& [site, bv] : lv.Bcol[a]) {
        const int64_t w = where(site);
        if (w < 0) continue;
        for (int j = 0; j < beta; ++j) SmG[size_t(a) * beta + j] += bv * Cs[size_t(w) * beta + j];
      }
    for (int a = 0; a < beta; ++a)
      for (int j = 0; j < beta; ++j) Sm[size_t(a) * beta + j] = SmG[size_t(a) * beta + j] + (a == j ? H.gamma[a] : 0.0);
    std::vector<double> Sinv;
    if (!dense_inverse(Sm, beta, Sinv)) {
      err = "singular capacitance matrix Gamma + B^T C";
      return MGMC_ENOTSPD;
    }
    std::vector<double> Gs(size_t(ns) * beta, 0.0);
    parallel_for(ns, [&](int64_t rb, int64_t re) {
      for (int64_t r = rb; r < re; ++r)
        for (int j = 0; j < beta; ++j) {
          double acc = 0.0;
          for (int t = 0; t < beta; ++t) acc += Cs[size_t(r) * beta + t] * Sinv[size_t(t) * beta + j];
          Gs[size_t(r) * beta + j] = acc;
        }
    });
    lv.supp[dir] = std::move(rows);
    lv.C[dir] = std::move(Cs);
    lv.G[dir] = std::move(Gs);
    lv.SmG[dir] = std::move(SmG);
    lv.Sinv[dir] = std::move(Sinv);
  }
  return MGMC_OK;
}

mgmc_status coarsest(HostHierarchy& H, std::string& err) {
  const HostLevel& c = H.lv[0];
  const int64_t N0 = c.N;
  const int S = H.S;
  Geo g{H.dim, c.n, N0};
  std::vector<double> a(size_t(N0) * N0, 0.0);
  int i[3], d[3], j[3];
  for (int64_t r = 0; r < N0; ++r) {
    g.coords(r, i);
    for (int t = 0; t < S; ++t) {
      const double v = c.st[size_t(t) * N0 + r];
      if (v == 0.0) continue;
      stencil_delta(H.dim, H.R, t, d);
      bool in = true;
      for (int k = 0; k < H.dim; ++k) {
        j[k] = i[k] + d[k];
        if (j[k] < 1 || j[k] > c.n) in = false;
      }
      if (in) a[size_t(r) * N0 + g.lin(j)] += v;
    }
  }
  for (int b = 0; b < H.beta; ++b)
    for (const auto& [r1, v1] : c.Bcol[b])
      for (const auto& [r2, v2] : c.Bcol[b]) a[size_t(r1) * N0 + r2] += v1 * v2 / H.gamma[b];
  // U^T U = a, U upper triangular (row-major)
  std::vector<double> U(size_t(N0) * N0, 0.0);
  for (int64_t r = 0; r < N0; ++r) {
    double dsum = a[size_t(r) * N0 + r];
    for (int64_t k = 0; k < r; ++k) dsum -= U[size_t(k) * N0 + r] * U[size_t(k) * N0 + r];
    if (!(dsum > 0.0)) {
      err = "coarsest matrix is not positive definite";
      return MGMC_ENOTSPD;
    }
    const double ur = std::sqrt(dsum);
    U[size_t(r) * N0 + r] = ur;
    for (int64_t col = r + 1; col < N0; ++col) {
      double s = a[size_t(r) * N0 + col];
      for (int64_t k = 0; k < r; ++k) s -= U[size_t(k) * N0 + r] * U[size_t(k) * N0 + col];
      U[size_t(r) * N0 + col] = s / ur;
    }
  }
  // Uinv by back substitution, column by column: U X = I
  std::vector<double> Ui(size_t(N0) * N0, 0.0);
  for (int64_t e = 0; e < N0; ++e) {
    for (int64_t r = e; r >= 0; --r) {
      double s = (r == e) ? 1.0 : 0.0;
      for (int64_t k = r + 1; k <= e; ++k) s -= U[size_t(r) * N0 + k] * Ui[size_t(k) * N0 + e];
      Ui[size_t(r) * N0 + e] = s / U[size_t(r) * N0 + r];
    }
  }
  // K = Uinv Uinv^T = At_0^{-1}
  H.K.assign(size_t(N0) * N0, 0.0);
  for (int64_t r = 0; r < N0; ++r)
    for (int64_t col = 0; col < N0; ++col) {
      double s = 0.0;
      for (int64_t k = std::max(r, col); k < N0; ++k) s += Ui[size_t(r) * N0 + k] * Ui[size_t(col) * N0 + k];
      H.K[size_t(r) * N0 + col] = s;
    }
  H.Uinv = std::move(Ui);
  return MGMC_OK;
}

}  // namespace

int forward_colour(int dim, int nclass, int q) {
  if (nclass == 3) return q;
  return dim == 2 ? kFwd2[q] : kFwd3[q];
}

mgmc_status build_hierarchy(const mgmc_problem& p, const mgmc_obs* obs, HostHierarchy& H,
                            std::string& err) {
  H.dim = p.dim;
  H.op = p.op;
  H.R = p.op == MGMC_OP_SSL13 ? 2 : 1;
  H.S = 1;
  for (int k = 0; k < p.dim; ++k) H.S *= 2 * H.R + 1;
  H.ncolours = 1;
  for (int k = 0; k < p.dim; ++k) H.ncolours *= H.R + 1;
  H.omega = p.omega > 0.0 ? p.omega : 1.0;
  H.level0_lowrank = p.sampler == MGMC_SAMPLER_GIBBS || (p.sampler == MGMC_SAMPLER_MGMC && p.nu0 > 0);
  H.L = p.levels - 1;
  H.h = 1.0 / (p.n + 1);
  H.scale = p.scale > 0 ? p.scale : std::pow(H.h, p.dim);
  H.lv.assign(p.levels, HostLevel{});
  for (int l = H.L, nl = p.n; l >= 0; --l, nl = (nl - 1) / 2) {
    H.lv[l].n = nl;
    int64_t N = 1;
    for (int k = 0; k < p.dim; ++k) N *= nl;
    H.lv[l].N = N;
  }
  if (p.op == MGMC_OP_FEM_Q1)
    fem_q1_operator(p, H);
  else if (p.op == MGMC_OP_SSL13)
    ssl13_operator(p, H);
  else
    fine_operator(p, H);
  if (p.prolong_w && H.L >= 1) {
    const size_t cnt = size_t(H.lv[H.L - 1].N) * (p.dim == 2 ? 9 : 27);
    H.lv[H.L].wP.assign(p.prolong_w, p.prolong_w + cnt);
  }
  for (int l = H.L; l >= 1; --l) galerkin(H, l, H.lv[l - 1]);
  for (int l = 0; l <= H.L; ++l) {
    const HostLevel& lv = H.lv[l];
    const double* diag = lv.st.data() + size_t((H.S - 1) / 2) * lv.N;
    for (int64_t i = 0; i < lv.N; ++i)
      if (!(diag[i] > 0.0)) {
        err = "non-positive diagonal on level " + std::to_string(l);
        return MGMC_ENOTSPD;
      }
  }
  H.beta = obs ? obs->beta : 0;
  if (obs) {
    H.gamma.assign(obs->gamma, obs->gamma + obs->beta);
    HostLevel& f = H.lv[H.L];
    f.Bcol.assign(obs->beta, {});
    for (int j = 0; j < obs->beta; ++j) {
      std::map<int64_t, double> col;
      for (int64_t e = obs->ptr[j]; e < obs->ptr[j + 1]; ++e) col[obs->idx[e]] += obs->val[e];
      f.Bcol[j].assign(col.begin(), col.end());
    }
    for (int l = H.L; l >= 1; --l) restrict_observations(H, l, H.lv[l - 1]);
    for (int l = H.level0_lowrank ? 0 : 1; l <= H.L; ++l) {
      mgmc_status st = lowrank_level(H, l, err);
      if (st != MGMC_OK) return st;
    }
  }
  if (p.sampler == MGMC_SAMPLER_CHOLESKY) return band_cholesky(H, err);
  if (H.level0_lowrank) return MGMC_OK;
  return coarsest(H, err);
}

// Banded Cholesky At = U^T U of the single level, lexicographic order.  The
// band is the largest |i - j| of a non-zero of At (stencil reach, widened by
// the couplings B Gamma^{-1} B^T of each observation's sites).  Right-looking
// in panels of kPanel rows: a panel's rows are finished one by one (each
// updates the rest of the panel), then the panel's rank-kPanel update of the
// next `band` rows runs over host threads.
mgmc_status band_cholesky(HostHierarchy& H, std::string& err) {
  const HostLevel& lv = H.lv[H.L];
  const int64_t N = lv.N;
  const int dim = H.dim, R = H.R, S = H.S;
  Geo g{dim, lv.n, N};
  int64_t band = 0;
  int dvec[3], iv[3];
  for (int t = 0; t < S; ++t) {
    stencil_delta(dim, R, t, dvec);
    int64_t off = 0, m = 1;
    for (int k = 0; k < dim; ++k) {
      off += dvec[k] * m;
      m *= lv.n;
    }
    bool used = false;
    for (int64_t i = 0; i < N && !used; ++i) used = lv.st[size_t(t) * N + i] != 0.0;
    if (used) band = std::max(band, off < 0 ? -off : off);
  }
  for (int j = 0; j < H.beta; ++j)
    if (!lv.Bcol[j].empty()) band = std::max(band, lv.Bcol[j].back().first - lv.Bcol[j].front().first);
  const int64_t W = band + 1;
  if (N * W > (int64_t(1) << 31)) {
    err = "banded factor exceeds 2^31 entries";
    return MGMC_EUNSUPPORTED;
  }
  std::vector<double> U(size_t(N) * W, 0.0);
  for (int64_t i = 0; i < N; ++i) {
    g.coords(i, iv);
    for (int t = 0; t < S; ++t) {
      const double v = lv.st[size_t(t) * N + i];
      if (v == 0.0) continue;
      stencil_delta(dim, R, t, dvec);
      int jv[3];
      bool in = true;
      for (int k = 0; k < dim; ++k) {
        jv[k] = iv[k] + dvec[k];
        if (jv[k] < 1 || jv[k] > lv.n) in = false;
      }
      if (!in) continue;
      const int64_t j = g.lin(jv);
      if (j >= i) U[size_t(i) * W + (j - i)] += v;
    }
  }
  for (int b = 0; b < H.beta; ++b)
    for (const auto& [r1, v1] : lv.Bcol[b])
      for (const auto& [r2, v2] : lv.Bcol[b])
        if (r2 >= r1) U[size_t(r1) * W + (r2 - r1)] += v1 * v2 / H.gamma[b];
  constexpr int64_t kPanel = 32;
  for (int64_t p0 = 0; p0 < N; p0 += kPanel) {
    const int64_t p1 = std::min(N, p0 + kPanel);
    for (int64_t i = p0; i < p1; ++i) {
      double* ui = &U[size_t(i) * W];
      if (!(ui[0] > 0.0)) {
        err = "single-level matrix At is not positive definite";
        return MGMC_ENOTSPD;
      }
      const double d = std::sqrt(ui[0]);
      ui[0] = d;
      const double id = 1.0 / d;
      for (int64_t k = 1; k < W; ++k) ui[k] *= id;
      // rows i+1 .. p1-1 of the panel
      for (int64_t j = i + 1; j < p1 && j - i < W; ++j) {
        const double uij = ui[j - i];
        if (uij == 0.0) continue;
        double* uj = &U[size_t(j) * W];
        for (int64_t k = j; k - i < W; ++k) uj[k - j] -= uij * ui[k - i];
      }
    }
    // rank-(p1 - p0) update of rows p1 .. p1 + band - 1
    const int64_t r0 = p1, r1 = std::min(N, p1 + band);
    parallel_for(r1 - r0, [&](int64_t b0, int64_t e0) {
      for (int64_t j = r0 + b0; j < r0 + e0; ++j) {
        double* uj = &U[size_t(j) * W];
        for (int64_t i = p0; i < p1; ++i) {
          if (j - i >= W) continue;
          const double* ui = &U[size_t(i) * W];
          const double uij = ui[j - i];
          if (uij == 0.0) continue;
          const int64_t kend = std::min(N, i + W);
          for (int64_t k = j; k < kend; ++k) uj[k - j] -= uij * ui[k - i];
        }
      }
    });
  }
  H.band = band;
  H.Uband = std::move(U);
  return MGMC_OK;
}

std::vector<double> band_solve(const HostHierarchy& H, const double* f) {
  const int64_t N = H.lv[H.L].N, W = H.band + 1;
  const std::vector<double>& U = H.Uband;
  std::vector<double> g(size_t(N), 0.0);
  // U^T g = f (U^T lower triangular): column-oriented forward substitution
  for (int64_t i = 0; i < N; ++i) g[size_t(i)] = f ? f[i] : 0.0;
  for (int64_t i = 0; i < N; ++i) {
    const double* ui = &U[size_t(i) * W];
    g[size_t(i)] /= ui[0];
    const double gi = g[size_t(i)];
    for (int64_t k = 1; k < W && i + k < N; ++k) g[size_t(i + k)] -= ui[k] * gi;
  }
  // U mu = g: row-oriented back substitution
  for (int64_t i = N - 1; i >= 0; --i) {
    const double* ui = &U[size_t(i) * W];
    double s = g[size_t(i)];
    for (int64_t k = 1; k < W && i + k < N; ++k) s -= ui[k] * g[size_t(i + k)];
    g[size_t(i)] = s / ui[0];
  }
  return g;
}

std::vector<double> posterior_rhs(const HostHierarchy& H, const double* y) {
  const HostLevel& f = H.lv[H.L];
  std::vector<double> out(f.N, 0.0);
  for (int j = 0; j < H.beta; ++j)
    for (const auto& [site, b] : f.Bcol[j]) out[site] += b * (y[j] / H.gamma[j]);
  return out;
}

}  // namespace mgmc
