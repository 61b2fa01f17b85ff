// Structured construction of the MGMC hierarchy (host, FP64).
//
//  * fine operator: s (kappa^2 I - div(a grad)) by finite differences with face
//    coefficients and zero Dirichlet data (paper Sec. 5.1.1);
//  * prolongation: column J of P carries w_J(delta) at fine node 2J + delta,
//    multilinear by default (Sec. 3.1, Sec. 5.1.3 "Samplers");
//  * Galerkin coarse operators A_{l-1} = P^T A_l P and B_{l-1} = P^T B_l
//    (eq. A_ell_1_B_ell_1), assembled stencil-wise;
//  * low-rank smoother data C = M^{-1} B, S = Gamma + B^T C, G = C S^{-1}
//    (Alg. 3 with omega = 1, M = D + L in colour order);
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

inline int stencil_index(int dim, const int* d) {
  int t = 0, m = 1;
  for (int k = 0; k < dim; ++k) {
    t += (d[k] + 1) * m;
    m *= 3;
  }
  return t;
}

inline void stencil_delta(int dim, int t, int* d) {
  for (int k = 0; k < dim; ++k) {
    d[k] = t % 3 - 1;
    t /= 3;
  }
}

// Multilinear weight of offset delta, or the user's weight of coarse node J.
inline double pweight(const HostLevel& fine, int S, int dim, int64_t J, int t) {
  if (!fine.wP.empty()) return fine.wP[size_t(J) * S + t];
  int d[3];
  stencil_delta(dim, t, d);
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
          f.st[size_t(stencil_index(dim, d)) * f.N + lin] = -s * ih2 * ap;
        }
        if (i[k] > 1) {
          d[k] = -1;
          f.st[size_t(stencil_index(dim, d)) * f.N + lin] = -s * ih2 * am;
        }
      }
      f.st[size_t(centre) * f.N + lin] = s * p.kappa2 + s * ih2 * faces;
    }
  });
}

// A_c = P^T A_f P, stencil by stencil: for coarse node J, every fine node
// i = 2J + d1 in the support of column J couples through A_f to fine j, and j
// lies in the support of the columns K covering it.
void galerkin(const HostHierarchy& H, int lf, HostLevel& c) {
  const HostLevel& f = H.lv[lf];
  const int dim = H.dim, S = H.S, nf = f.n, nc = c.n;
  Geo gf{dim, nf, f.N}, gc{dim, nc, c.N};
  c.st.assign(size_t(S) * c.N, 0.0);
  parallel_for(c.N, [&](int64_t b, int64_t e) {
    int J[3], d1[3], d2[3], i[3], j[3], K[3], opts[3][2], dl[3][2], nopt[3];
    for (int64_t Jl = b; Jl < e; ++Jl) {
      gc.coords(Jl, J);
      for (int t1 = 0; t1 < S; ++t1) {
        stencil_delta(dim, t1, d1);
        for (int k = 0; k < dim; ++k) i[k] = 2 * J[k] + d1[k];
        const double w1 = pweight(f, S, dim, Jl, t1);
        if (w1 == 0.0) continue;
        const int64_t il = gf.lin(i);
        for (int t2 = 0; t2 < S; ++t2) {
          const double a = f.st[size_t(t2) * f.N + il];
          if (a == 0.0) continue;
          stencil_delta(dim, t2, d2);
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
            const double w2 = pweight(f, S, dim, gc.lin(K), stencil_index(dim, dd));
            c.st[size_t(stencil_index(dim, dk)) * c.N + Jl] += w1 * a * w2;
          }
        }
      }
    }
  });
}

// B_{l-1} = P^T B_l column by column.
void restrict_observations(const HostHierarchy& H, int lf, HostLevel& c) {
  const HostLevel& f = H.lv[lf];
  const int dim = H.dim, S = H.S, nc = c.n;
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
        acc[Kl] += pweight(f, S, dim, Kl, stencil_index(dim, dd)) * b;
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
  const int dim = H.dim, S = H.S, n = lv.n, beta = H.beta, nq = H.ncolours;
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
          lo[k] = std::max(1, lo[k] - (nq - 1));
          hi[k] = std::min(n, hi[k] + (nq - 1));
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
          const int colour = forward_colour(dim, dir == 0 ? qq : nq - 1 - qq);
          for (int64_t v = 0; v < vol; ++v) {
            int64_t r = v;
            int c = 0;
            for (int k = 0; k < dim; ++k) {
              i[k] = lo[k] + int(r % ext[k]);
              r /= ext[k];
              c |= (i[k] & 1) << k;
            }
            if (c != colour) continue;
            const int64_t il = g.lin(i);
            double s = b[v];
            for (int t = 0; t < S; ++t) {
              if (t == centre) continue;
              const double a = lv.st[size_t(t) * lv.N + il];
              if (a == 0.0) continue;
              stencil_delta(dim, t, d);
              int jn[3];
              bool in = true;
              for (int k = 0; k < dim; ++k) {
                jn[k] = i[k] + d[k];
                if (jn[k] < lo[k] || jn[k] > hi[k]) in = false;
              }
              if (in) s -= a * x[boxlin(jn)];
            }
            x[v] = s / lv.st[size_t(centre) * lv.N + il];
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
      stencil_delta(H.dim, t, d);
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

int forward_colour(int dim, int q) { return dim == 2 ? kFwd2[q] : kFwd3[q]; }

mgmc_status build_hierarchy(const mgmc_problem& p, const mgmc_obs* obs, HostHierarchy& H,
                            std::string& err) {
  H.dim = p.dim;
  H.S = p.dim == 2 ? 9 : 27;
  H.ncolours = 1 << p.dim;
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
  fine_operator(p, H);
  if (p.prolong_w && H.L >= 1) {
    const size_t cnt = size_t(H.lv[H.L - 1].N) * H.S;
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
    for (int l = 1; l <= H.L; ++l) {
      mgmc_status st = lowrank_level(H, l, err);
      if (st != MGMC_OK) return st;
    }
  }
  return coarsest(H, err);
}

std::vector<double> posterior_rhs(const HostHierarchy& H, const double* y) {
  const HostLevel& f = H.lv[H.L];
  std::vector<double> out(f.N, 0.0);
  for (int j = 0; j < H.beta; ++j)
    for (const auto& [site, b] : f.Bcol[j]) out[site] += b * (y[j] / H.gamma[j]);
  return out;
}

}  // namespace mgmc
