/*
 * mgmc_oracle.c -- plain FP64 CPU reference of Multigrid Monte Carlo.
 *
 * TEST INFRASTRUCTURE ONLY (see mgmc_oracle.h).  Parity of every function
 * here is pinned by the CPU test-suite against closed forms, exact linear
 * algebra identities and published known-answer values; the references are
 * given per function.
 *
 * Conventions (paper Sec. 5.1.1, Sec. 2.3):
 *   sites are interior grid nodes i = (i_1..i_d), 1 <= i_k <= n, with zero
 *   Dirichlet values at i_k = 0 and n+1; linear index (i_1-1) + n (i_2-1) +
 *   n^2 (i_3-1); level 0 is the coarsest, level L = levels-1 the finest,
 *   n_{l-1} = (n_l - 1)/2 and coarse node J sits at fine node 2J.
 */
#include "mgmc_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static _Thread_local char g_err[256];
static void set_err(const char* msg) { snprintf(g_err, sizeof g_err, "%s", msg); }
const char* ora_last_error(void) { return g_err; }

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 and Box-Muller                                              */
/* ------------------------------------------------------------------------ */

/* Multipliers and Weyl increments of Philox4x32 as published by Salmon et al.
 * (SC'11, Sec. 3.3 / Table 2). */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    uint64_t prod0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
    uint64_t prod1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
    uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    x0 = y0;
    x1 = lo1;
    x2 = y2;
    x3 = lo0;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

static double uniform53(uint32_t hi, uint32_t lo) {
  uint64_t w = ((uint64_t)hi << 32) | (uint64_t)lo;
  return ((double)(w >> 11) + 0.5) * 0x1p-53;
}

void ora_normal_pair(const uint32_t ctr[4], const uint32_t key[2], double out[2]) {
  uint32_t x[4];
  ora_philox4x32_10(ctr, key, x);
  double u1 = uniform53(x[0], x[1]);
  double u2 = uniform53(x[2], x[3]);
  double radius = sqrt(-2.0 * log(u1));
  double angle = 6.283185307179586476925 * u2;
  out[0] = radius * cos(angle);
  out[1] = radius * sin(angle);
}

/* ------------------------------------------------------------------------ */
/* Generic CSR sparse matrices                                               */
/* ------------------------------------------------------------------------ */

typedef struct {
  int64_t nr, nc;
  int64_t* ptr;
  int32_t* col;
  double* val;
} csr;

static void csr_free(csr* m) {
  free(m->ptr);
  free(m->col);
  free(m->val);
  memset(m, 0, sizeof *m);
}

static void sort_row(int32_t* col, double* val, int64_t len) {
  for (int64_t a = 1; a < len; ++a) {
    int32_t c = col[a];
    double v = val[a];
    int64_t b = a - 1;
    while (b >= 0 && col[b] > c) {
      col[b + 1] = col[b];
      val[b + 1] = val[b];
      --b;
    }
    col[b + 1] = c;
    val[b + 1] = v;
  }
}

/* Build CSR from coordinate triplets; duplicates are summed. */
static int csr_from_coo(csr* m, int64_t nr, int64_t nc, int64_t nnz, const int64_t* ri,
                        const int32_t* ci, const double* vi) {
  m->nr = nr;
  m->nc = nc;
  m->ptr = calloc((size_t)nr + 1, sizeof(int64_t));
  m->col = malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
  m->val = malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(double));
  if (!m->ptr || !m->col || !m->val) return -1;
  for (int64_t e = 0; e < nnz; ++e) m->ptr[ri[e] + 1]++;
  for (int64_t r = 0; r < nr; ++r) m->ptr[r + 1] += m->ptr[r];
  int64_t* fill = malloc((size_t)(nr > 0 ? nr : 1) * sizeof(int64_t));
  if (!fill) return -1;
  for (int64_t r = 0; r < nr; ++r) fill[r] = m->ptr[r];
  for (int64_t e = 0; e < nnz; ++e) {
    int64_t at = fill[ri[e]]++;
    m->col[at] = ci[e];
    m->val[at] = vi[e];
  }
  free(fill);
  /* sort each row by column and merge duplicates */
  int64_t out = 0;
  int64_t start = 0;
  for (int64_t r = 0; r < nr; ++r) {
    int64_t end = m->ptr[r + 1];
    sort_row(m->col + start, m->val + start, end - start);
    int64_t row_begin = out;
    for (int64_t e = start; e < end; ++e) {
      if (out > row_begin && m->col[out - 1] == m->col[e]) {
        m->val[out - 1] += m->val[e];
      } else {
        m->col[out] = m->col[e];
        m->val[out] = m->val[e];
        ++out;
      }
    }
    start = end;
    m->ptr[r + 1] = out;
  }
  return 0;
}

static int csr_transpose(const csr* a, csr* t) {
  int64_t nnz = a->ptr[a->nr];
  int64_t* ri = malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int64_t));
  int32_t* ci = malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
  if (!ri || !ci) return -1;
  for (int64_t r = 0; r < a->nr; ++r)
    for (int64_t e = a->ptr[r]; e < a->ptr[r + 1]; ++e) {
      ri[e] = a->col[e];
      ci[e] = (int32_t)r;
    }
  int rc = csr_from_coo(t, a->nc, a->nr, nnz, ri, ci, a->val);
  free(ri);
  free(ci);
  return rc;
}

/* C = A * B, row by row with a dense accumulator. */
static int csr_matmul(const csr* a, const csr* b, csr* c) {
  double* acc = calloc((size_t)b->nc, sizeof(double));
  char* mark = calloc((size_t)b->nc, 1);
  int32_t* touched = malloc((size_t)b->nc * sizeof(int32_t));
  int64_t cap = a->ptr[a->nr] * 4 + 16, nnz = 0;
  int64_t* ri = malloc((size_t)cap * sizeof(int64_t));
  int32_t* ci = malloc((size_t)cap * sizeof(int32_t));
  double* vi = malloc((size_t)cap * sizeof(double));
  if (!acc || !mark || !touched || !ri || !ci || !vi) return -1;
  for (int64_t r = 0; r < a->nr; ++r) {
    int64_t nt = 0;
    for (int64_t e = a->ptr[r]; e < a->ptr[r + 1]; ++e) {
      int32_t k = a->col[e];
      double av = a->val[e];
      for (int64_t f = b->ptr[k]; f < b->ptr[k + 1]; ++f) {
        int32_t j = b->col[f];
        if (!mark[j]) {
          mark[j] = 1;
          touched[nt++] = j;
        }
        acc[j] += av * b->val[f];
      }
    }
    if (nnz + nt > cap) {
      cap = 2 * (nnz + nt) + 16;
      ri = realloc(ri, (size_t)cap * sizeof(int64_t));
      ci = realloc(ci, (size_t)cap * sizeof(int32_t));
      vi = realloc(vi, (size_t)cap * sizeof(double));
      if (!ri || !ci || !vi) return -1;
    }
    for (int64_t t = 0; t < nt; ++t) {
      int32_t j = touched[t];
      ri[nnz] = r;
      ci[nnz] = j;
      vi[nnz] = acc[j];
      ++nnz;
      acc[j] = 0.0;
      mark[j] = 0;
    }
  }
  int rc = csr_from_coo(c, a->nr, b->nc, nnz, ri, ci, vi);
  free(acc);
  free(mark);
  free(touched);
  free(ri);
  free(ci);
  free(vi);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Problem hierarchy                                                         */
/* ------------------------------------------------------------------------ */

typedef struct {
  int n;
  int64_t N;
  csr A;        /* prior operator A_l */
  double* diag; /* A_ii */
  csr P, PT;    /* prolongation from level l-1 (only l >= 1) */
  csr B, BT;    /* B_l (N x beta) and its transpose */
  uint8_t* colour;
  uint32_t* pair;
  uint8_t* slot;
  int32_t* order;      /* sites in forward colour order */
  int64_t cstart[10];  /* order[cstart[q] .. cstart[q+1]) has colour fwd_order[q] */
  int64_t nsupp[2];    /* rows where C_dir (hence G_dir) can be non-zero */
  int32_t* supp[2];
  double* G[2];        /* nsupp x beta, row-major */
} level;

struct ora_problem {
  int dim, n, L, nu1, nu2, ncolours;
  int q;        /* colour classes per axis: 2 for 3^d-point stencils, 3 for 5^d-point */
  int op;       /* fine operator: ORA_OP_FD, ORA_OP_FEM_Q1, ORA_OP_SSL13 */
  int cycle_gamma; /* recursive calls made by levels below the finest (Alg. 1) */
  int nu0;      /* 0: exact coarsest sample; k >= 1: Alg. 5 with k symmetric sweeps */
  int sampler;  /* ORA_SAMPLER_MGMC or ORA_SAMPLER_GIBBS */
  double omega; /* SOR relaxation of the Gibbs smoother (Sec. 3.3, 3.4) */
  double kappa2, scale, h;
  uint32_t seed_lo;
  level* lv;
  int beta;
  double* gamma;
  double* fL;
  double* U; /* coarsest Cholesky factor, upper triangular, row-major n0 x n0 */
  int noise_mode;
  int64_t impulse, drawn;
  uint32_t* noise_log; /* test hook: 7 words per draw (key, counter, slot) */
  int64_t noise_log_cap, noise_log_len;
  double restrict_scale; /* 1 in the method; other values only in planted-mistake tests */
};

/* Forward colour orders: colour id c = sum_k (i_k mod 2) 2^k; colours with
 * even parity sum first, then odd, each ascending.  On 5/7-point stencils this
 * is red-black Gauss-Seidel. */
static const int FWD2[4] = {0, 3, 1, 2};
static const int FWD3[8] = {0, 3, 5, 6, 1, 2, 4, 7};

/* With three classes per axis (5 x 5 stencils, 2D) the nine colours
 * c = (i_1 mod 3) + 3 (i_2 mod 3) are swept in ascending order. */
static int fwd_colour(const ora_problem* p, int q) {
  if (p->q == 3) return q;
  return p->dim == 2 ? FWD2[q] : FWD3[q];
}

static void coords(int dim, int n, int64_t lin, int* i) {
  for (int k = 0; k < dim; ++k) {
    i[k] = 1 + (int)(lin % n);
    lin /= n;
  }
}

static int64_t linear(int dim, int n, const int* i) {
  int64_t lin = 0;
  for (int k = dim - 1; k >= 0; --k) lin = lin * n + (i[k] - 1);
  return lin;
}

static double face_value(const ora_problem* p, const double* face, int k, const int* i, int fk) {
  if (!face) return 1.0;
  int n = p->n;
  int64_t per = (int64_t)(n + 1);
  for (int j = 1; j < p->dim; ++j) per *= n;
  int64_t idx = 0, mult = 1;
  for (int j = 0; j < p->dim; ++j) {
    int e = (j == k) ? n + 1 : n;
    int v = (j == k) ? fk : i[j] - 1;
    idx += (int64_t)v * mult;
    mult *= e;
  }
  return face[(int64_t)k * per + idx];
}

/* Lowest-order conforming (bilinear, Q1) finite elements of Sec. 5.1.1 for
 * -Laplace + kappa^2 on the uniform grid of n x n interior nodes, assembled
 * cell by cell from the element matrices of a square of side h (nodes in
 * counter-clockwise order from the lower left):
 *   stiffness  (1/6) [4 -1 -2 -1; -1 4 -1 -2; -2 -1 4 -1; -1 -2 -1 4],
 *   mass       (h^2/36) [4 2 1 2; 2 4 2 1; 1 2 4 2; 2 1 2 4];
 * rows and columns of boundary nodes are dropped (u = 0 there).  The result
 * is scaled by s / h^2, so the default s = h^2 gives the Galerkin matrix of
 * the bilinear form itself (eq. def-A_ell). */
static int build_fem_q1(ora_problem* p) {
  level* f = &p->lv[p->L];
  int n = p->n;
  int64_t cap = (int64_t)(n + 1) * (n + 1) * 16, nnz = 0;
  int64_t* ri = malloc((size_t)cap * sizeof(int64_t));
  int32_t* ci = malloc((size_t)cap * sizeof(int32_t));
  double* vi = malloc((size_t)cap * sizeof(double));
  if (!ri || !ci || !vi) return -1;
  static const double KE[4][4] = {{4, -1, -2, -1}, {-1, 4, -1, -2}, {-2, -1, 4, -1}, {-1, -2, -1, 4}};
  static const double ME[4][4] = {{4, 2, 1, 2}, {2, 4, 2, 1}, {1, 2, 4, 2}, {2, 1, 2, 4}};
  static const int CX[4] = {0, 1, 1, 0}, CY[4] = {0, 0, 1, 1};
  double h = p->h, sc = p->scale / (h * h);
  for (int cy = 0; cy <= n; ++cy)
    for (int cx = 0; cx <= n; ++cx) {
      /* cell with lower-left node (cx, cy); nodes 0..n+1 per axis */
      for (int a = 0; a < 4; ++a) {
        int ia[2] = {cx + CX[a], cy + CY[a]};
        if (ia[0] < 1 || ia[0] > n || ia[1] < 1 || ia[1] > n) continue;
        for (int b = 0; b < 4; ++b) {
          int ib[2] = {cx + CX[b], cy + CY[b]};
          if (ib[0] < 1 || ib[0] > n || ib[1] < 1 || ib[1] > n) continue;
          double v = KE[a][b] / 6.0 + p->kappa2 * (h * h) * ME[a][b] / 36.0;
          ri[nnz] = linear(2, n, ia);
          ci[nnz] = (int32_t)linear(2, n, ib);
          vi[nnz] = sc * v;
          ++nnz;
        }
      }
    }
  int rc = csr_from_coo(&f->A, f->N, f->N, nnz, ri, ci, vi);
  free(ri);
  free(ci);
  free(vi);
  return rc;
}

/* Squared shifted Laplace (Sec. 5.1.1, eq. squared_shifted_laplace),
 * (-Laplace + kappa^2)^2 = Laplace^2 - 2 kappa^2 Laplace + kappa^4, 2D:
 *   s [ h^-4 (13-point biharmonic stencil) + 2 kappa^2 h^-2 (5-point -Laplace)
 *       + kappa^4 ],
 * the biharmonic stencil with weight 20 at the centre, -8 at the four axis
 * neighbours, 2 at the four diagonal neighbours and 1 at the four nodes two
 * steps along an axis (Bjorstad's 13-point difference).  Boundary
 * conditions u = 0 and du/dn = 0 (clamped): nodes on the boundary are zero,
 * and the ghost node one step outside the boundary takes the value of its
 * mirror image inside (central difference of du/dn = 0), so a reach past the
 * boundary adds its weight to the interior mirror node. */
static int build_ssl13(ora_problem* p) {
  level* f = &p->lv[p->L];
  int n = p->n;
  int64_t N = f->N, cap = N * 13 + N * 5 + N, nnz = 0;
  int64_t* ri = malloc((size_t)cap * sizeof(int64_t));
  int32_t* ci = malloc((size_t)cap * sizeof(int32_t));
  double* vi = malloc((size_t)cap * sizeof(double));
  if (!ri || !ci || !vi) return -1;
  static const int OFF[13][2] = {{0, 0},  {1, 0},  {-1, 0}, {0, 1},  {0, -1}, {1, 1},  {1, -1},
                                 {-1, 1}, {-1, -1}, {2, 0},  {-2, 0}, {0, 2},  {0, -2}};
  static const double WB[13] = {20, -8, -8, -8, -8, 2, 2, 2, 2, 1, 1, 1, 1};
  double s = p->scale, h = p->h, ih2 = 1.0 / (h * h), ih4 = ih2 * ih2, k2 = p->kappa2;
  int i[2], j[2];
  for (int64_t lin = 0; lin < N; ++lin) {
    coords(2, n, lin, i);
    for (int t = 0; t < 13; ++t) {
      int skip = 0;
      for (int k = 0; k < 2; ++k) {
        j[k] = i[k] + OFF[t][k];
        if (j[k] == 0 || j[k] == n + 1) skip = 1;   /* boundary node: u = 0 */
        if (j[k] == -1) j[k] = 1;                   /* mirror of the ghost node */
        if (j[k] == n + 2) j[k] = n;
      }
      if (skip) continue;
      ri[nnz] = lin; ci[nnz] = (int32_t)linear(2, n, j); vi[nnz] = s * ih4 * WB[t]; ++nnz;
    }
    for (int t = 0; t < 5; ++t) {
      int skip = 0;
      for (int k = 0; k < 2; ++k) {
        j[k] = i[k] + OFF[t][k];
        if (j[k] < 1 || j[k] > n) skip = 1;
      }
      if (skip) continue;
      double w = (t == 0) ? 4.0 : -1.0;
      ri[nnz] = lin; ci[nnz] = (int32_t)linear(2, n, j); vi[nnz] = s * 2.0 * k2 * ih2 * w; ++nnz;
    }
    ri[nnz] = lin; ci[nnz] = (int32_t)lin; vi[nnz] = s * k2 * k2; ++nnz;
  }
  int rc = csr_from_coo(&f->A, N, N, nnz, ri, ci, vi);
  free(ri);
  free(ci);
  free(vi);
  return rc;
}

/* Finite-difference operator of Sec. 5.1.1 in divergence form with face
 * coefficients: (A u)_i = s [kappa^2 u_i + h^-2 sum_k a_{i+e_k/2}(u_i - u_{i+e_k})
 * + a_{i-e_k/2}(u_i - u_{i-e_k})], u = 0 outside the interior. */
static int build_fine_operator(ora_problem* p, const double* face) {
  level* f = &p->lv[p->L];
  int d = p->dim, n = p->n;
  int64_t N = f->N, cap = N * (2 * d + 1), nnz = 0;
  int64_t* ri = malloc((size_t)cap * sizeof(int64_t));
  int32_t* ci = malloc((size_t)cap * sizeof(int32_t));
  double* vi = malloc((size_t)cap * sizeof(double));
  if (!ri || !ci || !vi) return -1;
  double s = p->scale, ih2 = 1.0 / (p->h * p->h);
  int i[3];
  for (int64_t lin = 0; lin < N; ++lin) {
    coords(d, n, lin, i);
    double faces = 0.0;
    int64_t stride = 1;
    for (int k = 0; k < d; ++k) {
      double ap = face_value(p, face, k, i, i[k]);
      double am = face_value(p, face, k, i, i[k] - 1);
      faces += ap + am;
      if (i[k] < n) {
        ri[nnz] = lin; ci[nnz] = (int32_t)(lin + stride); vi[nnz] = -s * ih2 * ap; ++nnz;
      }
      if (i[k] > 1) {
        ri[nnz] = lin; ci[nnz] = (int32_t)(lin - stride); vi[nnz] = -s * ih2 * am; ++nnz;
      }
      stride *= n;
    }
    ri[nnz] = lin; ci[nnz] = (int32_t)lin; vi[nnz] = s * (p->kappa2 + ih2 * faces); ++nnz;
  }
  int rc = csr_from_coo(&f->A, N, N, nnz, ri, ci, vi);
  free(ri);
  free(ci);
  free(vi);
  return rc;
}

/* Canonical prolongation (Sec. 3.1): column J of P carries weight w_J(delta)
 * at fine node 2J + delta, delta in {-1,0,1}^d; multilinear interpolation has
 * w = prod_k (1 if delta_k = 0 else 1/2).  User weights replace w on the
 * finest transfer. */
static int build_prolongation(ora_problem* p, int l, const double* user_w) {
  level* fine = &p->lv[l];
  level* coarse = &p->lv[l - 1];
  int d = p->dim, nc = coarse->n, nf = fine->n;
  int stencil = (d == 2) ? 9 : 27;
  int64_t cap = coarse->N * stencil, nnz = 0;
  int64_t* ri = malloc((size_t)cap * sizeof(int64_t));
  int32_t* ci = malloc((size_t)cap * sizeof(int32_t));
  double* vi = malloc((size_t)cap * sizeof(double));
  if (!ri || !ci || !vi) return -1;
  int J[3], I[3], del[3];
  for (int64_t jl = 0; jl < coarse->N; ++jl) {
    coords(d, nc, jl, J);
    for (int t = 0; t < stencil; ++t) {
      int rem = t;
      double w = 1.0;
      for (int k = 0; k < d; ++k) {
        del[k] = rem % 3 - 1;
        rem /= 3;
        I[k] = 2 * J[k] + del[k];
        if (del[k] != 0) w *= 0.5;
      }
      if (user_w) w = user_w[jl * stencil + t];
      ri[nnz] = linear(d, nf, I);
      ci[nnz] = (int32_t)jl;
      vi[nnz] = w;
      ++nnz;
    }
  }
  int rc = csr_from_coo(&fine->P, fine->N, coarse->N, nnz, ri, ci, vi);
  if (rc == 0) rc = csr_transpose(&fine->P, &fine->PT);
  free(ri);
  free(ci);
  free(vi);
  return rc;
}

static int build_colouring(ora_problem* p, int l) {
  level* lv = &p->lv[l];
  int d = p->dim, n = lv->n;
  int64_t N = lv->N;
  lv->colour = malloc((size_t)N);
  lv->pair = malloc((size_t)N * sizeof(uint32_t));
  lv->slot = malloc((size_t)N);
  lv->order = malloc((size_t)N * sizeof(int32_t));
  lv->diag = malloc((size_t)N * sizeof(double));
  if (!lv->colour || !lv->pair || !lv->slot || !lv->order || !lv->diag) return -1;
  int i[3];
  int q = p->q;
  for (int64_t lin = 0; lin < N; ++lin) {
    coords(d, n, lin, i);
    int c = 0, mult = 1;
    int s[3] = {0, 0, 0}, m[3] = {1, 1, 1};
    for (int k = 0; k < d; ++k) {
      /* class of the axis coordinate, position in its sublattice, and the
       * number of coordinates 1..n in the class */
      int par = i[k] % q;
      int first = par == 0 ? q : par;
      c += par * mult;
      mult *= q;
      s[k] = (i[k] - 1) / q;
      m[k] = first <= n ? (n - first) / q + 1 : 0;
    }
    lv->colour[lin] = (uint8_t)c;
    lv->pair[lin] = (uint32_t)((s[0] >> 1) + (int64_t)((m[0] + 1) / 2) * (s[1] + (int64_t)m[1] * s[2]));
    lv->slot[lin] = (uint8_t)(s[0] & 1);
  }
  int64_t at = 0;
  for (int q = 0; q < p->ncolours; ++q) {
    int c = fwd_colour(p, q);
    lv->cstart[q] = at;
    for (int64_t lin = 0; lin < N; ++lin)
      if (lv->colour[lin] == c) lv->order[at++] = (int32_t)lin;
  }
  lv->cstart[p->ncolours] = at;
  /* Diagonal, and the check that same-coloured sites never couple, which is
   * what makes the colour-ordered sweep a Gauss-Seidel sweep for M = D + L. */
  for (int64_t r = 0; r < N; ++r) {
    lv->diag[r] = 0.0;
    for (int64_t e = lv->A.ptr[r]; e < lv->A.ptr[r + 1]; ++e) {
      int32_t c = lv->A.col[e];
      if (c == r) {
        lv->diag[r] = lv->A.val[e];
      } else if (lv->colour[c] == lv->colour[r] && lv->A.val[e] != 0.0) {
        set_err("same-coloured sites are coupled");
        return -1;
      }
    }
    if (!(lv->diag[r] > 0.0)) {
      set_err("non-positive diagonal");
      return -1;
    }
  }
  return 0;
}

static void free_level(level* lv) {
  csr_free(&lv->A);
  csr_free(&lv->P);
  csr_free(&lv->PT);
  csr_free(&lv->B);
  csr_free(&lv->BT);
  free(lv->diag);
  free(lv->colour);
  free(lv->pair);
  free(lv->slot);
  free(lv->order);
  for (int d = 0; d < 2; ++d) {
    free(lv->supp[d]);
    free(lv->G[d]);
  }
}

void ora_destroy(ora_problem* p) {
  if (!p) return;
  if (p->lv)
    for (int l = 0; l <= p->L; ++l) free_level(&p->lv[l]);
  free(p->lv);
  free(p->gamma);
  free(p->fL);
  free(p->U);
  free(p);
}

/* Dense coarsest matrix At_0 = A_0 + B_0 Gamma^{-1} B_0^T (eq. galerkin_triple_product). */
static double* dense_tilde(const ora_problem* p, int l) {
  const level* lv = &p->lv[l];
  int64_t N = lv->N;
  double* a = calloc((size_t)(N * N), sizeof(double));
  if (!a) return NULL;
  for (int64_t r = 0; r < N; ++r)
    for (int64_t e = lv->A.ptr[r]; e < lv->A.ptr[r + 1]; ++e) a[r * N + lv->A.col[e]] += lv->A.val[e];
  for (int j = 0; j < p->beta; ++j)
    for (int64_t e = lv->BT.ptr[j]; e < lv->BT.ptr[j + 1]; ++e)
      for (int64_t f = lv->BT.ptr[j]; f < lv->BT.ptr[j + 1]; ++f)
        a[(int64_t)lv->BT.col[e] * N + lv->BT.col[f]] += lv->BT.val[e] * lv->BT.val[f] / p->gamma[j];
  return a;
}

/* Textbook Cholesky At_0 = U^T U with U upper triangular (Sec. 5.1.3). */
static int coarse_cholesky(ora_problem* p) {
  int64_t n0 = p->lv[0].N;
  double* a = dense_tilde(p, 0);
  if (!a) return -1;
  free(p->U);
  p->U = calloc((size_t)(n0 * n0), sizeof(double));
  if (!p->U) return -1;
  double* U = p->U;
  for (int64_t i = 0; i < n0; ++i) {
    double s = a[i * n0 + i];
    for (int64_t k = 0; k < i; ++k) s -= U[k * n0 + i] * U[k * n0 + i];
    if (!(s > 0.0)) {
      free(a);
      set_err("coarsest matrix is not positive definite");
      return -2;
    }
    U[i * n0 + i] = sqrt(s);
    for (int64_t j = i + 1; j < n0; ++j) {
      double t = a[i * n0 + j];
      for (int64_t k = 0; k < i; ++k) t -= U[k * n0 + i] * U[k * n0 + j];
      U[i * n0 + j] = t / U[i * n0 + i];
    }
  }
  free(a);
  return 0;
}

ora_problem* ora_create_ex(const ora_options* o) {
  int dim = o->dim, n = o->n, levels = o->levels, nu1 = o->nu1, nu2 = o->nu2;
  g_err[0] = 0;
  if (dim != 2 && dim != 3) { set_err("dim must be 2 or 3"); return NULL; }
  if (n < 1 || ((n + 1) & n) != 0) { set_err("n must be 2^k - 1"); return NULL; }
  int k = 0;
  while ((1 << k) < n + 1) ++k;
  if (levels < 1 || levels > k) { set_err("levels out of range"); return NULL; }
  if (nu1 < 1 || nu2 < 1 || nu1 + nu2 > 16) { set_err("nu1, nu2 out of range"); return NULL; }
  if (o->op < ORA_OP_FD || o->op > ORA_OP_SSL13) { set_err("unknown operator"); return NULL; }
  if (o->op != ORA_OP_FD && (dim != 2 || o->face_coef)) {
    set_err("the FEM and squared shifted Laplace operators are 2D with a = 1");
    return NULL;
  }
  double omega = o->omega > 0.0 ? o->omega : 1.0;
  if (!(omega < 2.0)) { set_err("omega must lie in (0, 2)"); return NULL; }
  int gamma = o->gamma > 0 ? o->gamma : 1;
  if (gamma > 3 || o->nu0 < 0 || o->nu0 > 8) { set_err("gamma or nu0 out of range"); return NULL; }
  if (o->sampler == ORA_SAMPLER_GIBBS && levels != 1) { set_err("the Gibbs sampler runs on one level"); return NULL; }
  if (o->sampler != ORA_SAMPLER_MGMC && o->sampler != ORA_SAMPLER_GIBBS) { set_err("unknown sampler"); return NULL; }
  int n0 = ((n + 1) >> (levels - 1)) - 1;
  int64_t N0 = 1;
  for (int j = 0; j < dim; ++j) N0 *= n0;
  int exact_coarse = o->sampler == ORA_SAMPLER_MGMC && o->nu0 == 0;
  if (exact_coarse && N0 > 8192) { set_err("coarsest level too large for a dense factor"); return NULL; }
  ora_problem* p = calloc(1, sizeof *p);
  if (!p) return NULL;
  p->dim = dim;
  p->n = n;
  p->L = levels - 1;
  p->nu1 = nu1;
  p->nu2 = nu2;
  p->op = o->op;
  p->q = o->op == ORA_OP_SSL13 ? 3 : 2;
  p->ncolours = dim == 2 ? p->q * p->q : 8;
  p->cycle_gamma = gamma;
  p->nu0 = o->nu0;
  p->sampler = o->sampler;
  p->omega = omega;
  p->kappa2 = o->kappa2;
  p->h = 1.0 / (n + 1);
  p->scale = o->scale > 0.0 ? o->scale : pow(p->h, dim);
  p->seed_lo = (uint32_t)o->seed;
  p->restrict_scale = 1.0;
  p->lv = calloc((size_t)levels, sizeof(level));
  if (!p->lv) { free(p); return NULL; }
  for (int l = p->L, nl = n; l >= 0; --l, nl = (nl - 1) / 2) {
    p->lv[l].n = nl;
    int64_t N = 1;
    for (int j = 0; j < dim; ++j) N *= nl;
    p->lv[l].N = N;
  }
  int rc = o->op == ORA_OP_FEM_Q1 ? build_fem_q1(p)
           : o->op == ORA_OP_SSL13 ? build_ssl13(p)
                                   : build_fine_operator(p, o->face_coef);
  if (rc) goto fail;
  for (int l = p->L; l >= 1; --l) {
    if (build_prolongation(p, l, (l == p->L) ? o->prolong_w : NULL)) goto fail;
    /* Galerkin triple product A_{l-1} = P^T A_l P (eq. A_ell_1_B_ell_1). */
    csr AP;
    memset(&AP, 0, sizeof AP);
    if (csr_matmul(&p->lv[l].A, &p->lv[l].P, &AP)) goto fail;
    if (csr_matmul(&p->lv[l].PT, &AP, &p->lv[l - 1].A)) { csr_free(&AP); goto fail; }
    csr_free(&AP);
  }
  for (int l = 0; l <= p->L; ++l)
    if (build_colouring(p, l)) goto fail;
  if (exact_coarse && coarse_cholesky(p)) goto fail;
  return p;
fail:
  if (g_err[0] == 0) set_err("allocation failed");
  ora_destroy(p);
  return NULL;
}

ora_problem* ora_create(int dim, int n, int levels, double kappa2, double scale,
                        const double* face_coef, const double* prolong_w, int nu1, int nu2,
                        uint64_t seed) {
  ora_options o;
  memset(&o, 0, sizeof o);
  o.dim = dim;
  o.n = n;
  o.levels = levels;
  o.kappa2 = kappa2;
  o.scale = scale;
  o.face_coef = face_coef;
  o.prolong_w = prolong_w;
  o.nu1 = nu1;
  o.nu2 = nu2;
  o.seed = seed;
  return ora_create_ex(&o);
}

/* ------------------------------------------------------------------------ */
/* Observations and the low-rank smoother setup (Alg. 3)                     */
/* ------------------------------------------------------------------------ */

/* C = M^{-1} B for M = D/omega + L (forward) or D/omega + L^T (backward)
 * under the colour ordering (Alg. 3 setup, eq. Bellstar_definition), one column at a time by substitution in sweep order; rows where
 * any column is non-zero form the support of C and of G = C S^{-1}. */
static int lowrank_setup(ora_problem* p, int l, int dir) {
  level* lv = &p->lv[l];
  int beta = p->beta;
  int64_t N = lv->N;
  double* x = calloc((size_t)N, sizeof(double));
  double* b = calloc((size_t)N, sizeof(double));
  char* used = calloc((size_t)N, 1);
  /* column values are kept sparse: (row, value) lists per column */
  int64_t* cnt = calloc((size_t)beta, sizeof(int64_t));
  int32_t** rows = calloc((size_t)beta, sizeof(int32_t*));
  double** vals = calloc((size_t)beta, sizeof(double*));
  if (!x || !b || !used || !cnt || !rows || !vals) return -1;
  int nq = p->ncolours;
  for (int j = 0; j < beta; ++j) {
    memset(x, 0, (size_t)N * sizeof(double));
    memset(b, 0, (size_t)N * sizeof(double));
    for (int64_t e = lv->BT.ptr[j]; e < lv->BT.ptr[j + 1]; ++e) b[lv->BT.col[e]] = lv->BT.val[e];
    for (int qq = 0; qq < nq; ++qq) {
      int q = dir == 0 ? qq : nq - 1 - qq;
      for (int64_t t = lv->cstart[q]; t < lv->cstart[q + 1]; ++t) {
        int32_t i = lv->order[t];
        double s = b[i];
        for (int64_t e = lv->A.ptr[i]; e < lv->A.ptr[i + 1]; ++e)
          if (lv->A.col[e] != i) s -= lv->A.val[e] * x[lv->A.col[e]];
        x[i] = (p->omega * s) / lv->diag[i];
      }
    }
    int64_t c = 0;
    for (int64_t i = 0; i < N; ++i) c += (x[i] != 0.0);
    rows[j] = malloc((size_t)(c > 0 ? c : 1) * sizeof(int32_t));
    vals[j] = malloc((size_t)(c > 0 ? c : 1) * sizeof(double));
    if (!rows[j] || !vals[j]) return -1;
    cnt[j] = 0;
    for (int64_t i = 0; i < N; ++i)
      if (x[i] != 0.0) {
        rows[j][cnt[j]] = (int32_t)i;
        vals[j][cnt[j]] = x[i];
        cnt[j]++;
        used[i] = 1;
      }
  }
  int64_t ns = 0;
  for (int64_t i = 0; i < N; ++i) ns += used[i];
  int32_t* supp = malloc((size_t)(ns > 0 ? ns : 1) * sizeof(int32_t));
  int64_t* where = malloc((size_t)N * sizeof(int64_t));
  double* Cs = calloc((size_t)(ns * beta > 0 ? ns * beta : 1), sizeof(double));
  if (!supp || !where || !Cs) return -1;
  ns = 0;
  for (int64_t i = 0; i < N; ++i) {
    where[i] = -1;
    if (used[i]) {
      where[i] = ns;
      supp[ns++] = (int32_t)i;
    }
  }
  for (int j = 0; j < beta; ++j)
    for (int64_t t = 0; t < cnt[j]; ++t) Cs[where[rows[j][t]] * beta + j] = vals[j][t];
  /* S = Gamma + B^T C (Alg. 3), beta x beta, row-major */
  double* S = calloc((size_t)beta * beta, sizeof(double));
  double* Sinv = calloc((size_t)beta * beta, sizeof(double));
  int* piv = malloc((size_t)beta * sizeof(int));
  if (!S || !Sinv || !piv) return -1;
  for (int i = 0; i < beta; ++i) {
    for (int j = 0; j < beta; ++j) {
      double acc = 0.0;
      for (int64_t e = lv->BT.ptr[i]; e < lv->BT.ptr[i + 1]; ++e) {
        int64_t w = where[lv->BT.col[e]];
        if (w >= 0) acc += lv->BT.val[e] * Cs[w * beta + j];
      }
      S[i * beta + j] = acc + (i == j ? p->gamma[i] : 0.0);
    }
  }
  /* S^{-1} by LU with partial pivoting (S is not symmetric: M is triangular). */
  for (int c = 0; c < beta; ++c) piv[c] = c;
  for (int c = 0; c < beta; ++c) {
    int best = c;
    for (int r = c + 1; r < beta; ++r)
      if (fabs(S[r * beta + c]) > fabs(S[best * beta + c])) best = r;
    if (S[best * beta + c] == 0.0) { set_err("singular capacitance matrix"); return -1; }
    if (best != c) {
      for (int t = 0; t < beta; ++t) {
        double tmp = S[c * beta + t];
        S[c * beta + t] = S[best * beta + t];
        S[best * beta + t] = tmp;
      }
      int tp = piv[c]; piv[c] = piv[best]; piv[best] = tp;
    }
    for (int r = c + 1; r < beta; ++r) {
      double f = S[r * beta + c] / S[c * beta + c];
      S[r * beta + c] = f;
      for (int t = c + 1; t < beta; ++t) S[r * beta + t] -= f * S[c * beta + t];
    }
  }
  double* col = malloc((size_t)beta * sizeof(double));
  if (!col) return -1;
  for (int e = 0; e < beta; ++e) {
    for (int r = 0; r < beta; ++r) col[r] = (piv[r] == e) ? 1.0 : 0.0;
    for (int r = 0; r < beta; ++r)
      for (int t = 0; t < r; ++t) col[r] -= S[r * beta + t] * col[t];
    for (int r = beta - 1; r >= 0; --r) {
      for (int t = r + 1; t < beta; ++t) col[r] -= S[r * beta + t] * col[t];
      col[r] /= S[r * beta + r];
    }
    for (int r = 0; r < beta; ++r) Sinv[r * beta + e] = col[r];
  }
  /* G = C S^{-1} on the support rows (Alg. 3, eq. Bellstar_definition) */
  double* G = calloc((size_t)(ns * beta > 0 ? ns * beta : 1), sizeof(double));
  if (!G) return -1;
  for (int64_t r = 0; r < ns; ++r)
    for (int j = 0; j < beta; ++j) {
      double acc = 0.0;
      for (int t = 0; t < beta; ++t) acc += Cs[r * beta + t] * Sinv[t * beta + j];
      G[r * beta + j] = acc;
    }
  free(lv->supp[dir]);
  free(lv->G[dir]);
  lv->nsupp[dir] = ns;
  lv->supp[dir] = supp;
  lv->G[dir] = G;
  for (int j = 0; j < beta; ++j) {
    free(rows[j]);
    free(vals[j]);
  }
  free(rows); free(vals); free(cnt); free(used); free(x); free(b);
  free(where); free(Cs); free(S); free(Sinv); free(piv); free(col);
  return 0;
}

/* Level 0 is updated by Gibbs sweeps (Alg. 5, or the standalone Gibbs
 * sampler) rather than sampled exactly. */
static int smoothed_coarsest(const ora_problem* p) {
  return p->sampler == ORA_SAMPLER_GIBBS || p->nu0 > 0;
}

int ora_set_obs(ora_problem* p, int beta, const int64_t* ptr, const int32_t* idx,
                const double* val, const double* gamma) {
  if (!p || beta < 0 || (beta > 0 && (!ptr || !idx || !val || !gamma))) {
    set_err("invalid observation arguments");
    return -1;
  }
  for (int j = 0; j < beta; ++j)
    if (!(gamma[j] > 0.0)) { set_err("gamma must be positive"); return -1; }
  level* fine = &p->lv[p->L];
  for (int j = 0; j < beta; ++j)
    for (int64_t e = ptr[j]; e < ptr[j + 1]; ++e)
      if (idx[e] < 0 || idx[e] >= fine->N) { set_err("observation index out of range"); return -1; }
  p->beta = beta;
  free(p->gamma);
  p->gamma = malloc((size_t)(beta > 0 ? beta : 1) * sizeof(double));
  for (int j = 0; j < beta; ++j) p->gamma[j] = gamma[j];
  /* B_L (N_L x beta), then B_{l-1} = P^T B_l (eq. A_ell_1_B_ell_1) */
  int64_t nnz = beta > 0 ? ptr[beta] : 0;
  int64_t* ri = malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int64_t));
  int32_t* ci = malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
  if (!ri || !ci) return -1;
  for (int j = 0; j < beta; ++j)
    for (int64_t e = ptr[j]; e < ptr[j + 1]; ++e) {
      ri[e] = idx[e];
      ci[e] = j;
    }
  for (int l = 0; l <= p->L; ++l) {
    csr_free(&p->lv[l].B);
    csr_free(&p->lv[l].BT);
  }
  if (csr_from_coo(&fine->B, fine->N, beta, nnz, ri, ci, val)) return -1;
  free(ri);
  free(ci);
  for (int l = p->L; l >= 1; --l)
    if (csr_matmul(&p->lv[l].PT, &p->lv[l].B, &p->lv[l - 1].B)) return -1;
  for (int l = 0; l <= p->L; ++l)
    if (csr_transpose(&p->lv[l].B, &p->lv[l].BT)) return -1;
  int l0 = smoothed_coarsest(p) ? 0 : 1;
  for (int l = l0; l <= p->L; ++l)
    for (int dir = 0; dir < 2; ++dir)
      if (lowrank_setup(p, l, dir)) return -1;
  return smoothed_coarsest(p) ? 0 : coarse_cholesky(p);
}

void ora_set_rhs(ora_problem* p, const double* f) {
  free(p->fL);
  p->fL = NULL;
  if (!f) return;
  int64_t N = p->lv[p->L].N;
  p->fL = malloc((size_t)N * sizeof(double));
  memcpy(p->fL, f, (size_t)N * sizeof(double));
}

int ora_set_posterior_rhs(ora_problem* p, const double* y) {
  if (p->beta == 0) { set_err("no observations"); return -1; }
  level* fine = &p->lv[p->L];
  int64_t N = fine->N;
  free(p->fL);
  p->fL = calloc((size_t)N, sizeof(double));
  for (int j = 0; j < p->beta; ++j)
    for (int64_t e = fine->BT.ptr[j]; e < fine->BT.ptr[j + 1]; ++e)
      p->fL[fine->BT.col[e]] += fine->BT.val[e] * (y[j] / p->gamma[j]);
  return 0;
}

void ora_set_noise(ora_problem* p, int mode, int64_t impulse_index) {
  p->noise_mode = mode;
  p->impulse = impulse_index;
  p->drawn = 0;
}

int64_t ora_noise_drawn(const ora_problem* p) { return p->drawn; }

void ora_set_restriction_scale(ora_problem* p, double scale) { p->restrict_scale = scale; }

void ora_set_noise_log(ora_problem* p, uint32_t* buf, int64_t cap) {
  p->noise_log = buf;
  p->noise_log_cap = buf ? cap : 0;
  p->noise_log_len = 0;
}

int64_t ora_noise_log_len(const ora_problem* p) { return p->noise_log_len; }

/* ------------------------------------------------------------------------ */
/* The Markov update                                                         */
/* ------------------------------------------------------------------------ */

/* Noise stream.  Key = (seed low word, chain); counter = (pair, visit<<16 |
 * level<<8 | sweep<<4 | colour, sample index m, tag) with tag 0 site noise,
 * 1 the low-rank normals zeta_j, 2 the coarsest-level normals; visit is 0
 * except on coarse levels that a W-cycle calls more than once. */
static double draw(ora_problem* p, uint32_t chain, uint32_t m, uint32_t word1, uint32_t pair,
                   int slot, uint32_t tag) {
  if (p->noise_log) {
    if (p->noise_log_len < p->noise_log_cap) {
      uint32_t* e = p->noise_log + 7 * p->noise_log_len;
      e[0] = p->seed_lo;
      e[1] = chain;
      e[2] = pair;
      e[3] = word1;
      e[4] = m;
      e[5] = tag;
      e[6] = (uint32_t)slot;
    }
    p->noise_log_len++;
  }
  if (p->noise_mode == 1) {
    p->drawn++;
    return 0.0;
  }
  if (p->noise_mode == 2) {
    double v = (p->drawn == p->impulse) ? 1.0 : 0.0;
    p->drawn++;
    return v;
  }
  uint32_t ctr[4] = {pair, word1, m, tag};
  uint32_t key[2] = {p->seed_lo, chain};
  double z[2];
  ora_normal_pair(ctr, key, z);
  return z[slot];
}

typedef struct {
  double** theta; /* per level < L: psi */
  double** f;     /* per level < L: restricted rhs */
  double* g;      /* smoother rhs scratch (N_L) */
  double* r;      /* residual scratch (N_L) */
  double* w;      /* beta */
  double* t;      /* coarse scratch (N_0) */
  uint32_t* visits; /* per level: calls so far in the current update */
} workspace;

static void ws_free(workspace* ws, int L) {
  if (ws->theta)
    for (int l = 0; l < L; ++l) free(ws->theta[l]);
  if (ws->f)
    for (int l = 0; l < L; ++l) free(ws->f[l]);
  free(ws->theta);
  free(ws->f);
  free(ws->g);
  free(ws->r);
  free(ws->w);
  free(ws->t);
  free(ws->visits);
}

static int ws_alloc(const ora_problem* p, workspace* ws) {
  memset(ws, 0, sizeof *ws);
  int64_t NL = p->lv[p->L].N;
  ws->theta = calloc((size_t)p->L + 1, sizeof(double*));
  ws->f = calloc((size_t)p->L + 1, sizeof(double*));
  ws->g = malloc((size_t)NL * sizeof(double));
  ws->r = malloc((size_t)NL * sizeof(double));
  ws->w = malloc((size_t)(p->beta + 1) * sizeof(double));
  ws->t = malloc((size_t)p->lv[0].N * sizeof(double));
  ws->visits = calloc((size_t)p->L + 1, sizeof(uint32_t));
  if (!ws->theta || !ws->f || !ws->g || !ws->r || !ws->w || !ws->t || !ws->visits) return -1;
  for (int l = 0; l < p->L; ++l) {
    ws->theta[l] = malloc((size_t)p->lv[l].N * sizeof(double));
    ws->f[l] = malloc((size_t)p->lv[l].N * sizeof(double));
    if (!ws->theta[l] || !ws->f[l]) return -1;
  }
  return 0;
}

/* Gibbs smoother with low-rank correction (Alg. 3), SOR relaxation omega:
 *   g = f + B xi_LR, xi_LR = Gamma^{-1/2} zeta;
 *   theta* = theta + M^{-1}(g + sqrt((2-omega)/omega) xi_diag - A theta),
 *     M = D/omega + L, xi_diag ~ N(0, D), done as the in-place colour-ordered
 *     SOR substitution
 *     theta_i = (1-omega) theta_i + omega (g_i - sum_{j != i} A_ij theta_j)/A_ii
 *               + sqrt(omega (2-omega) / A_ii) z_i
 *     (omega = 1: theta_i = (g_i - sum ...)/A_ii + z_i/sqrt(A_ii));
 *   theta' = theta* - G (B^T theta*).
 * Without observations it is the plain random Gibbs / SOR sweep (Alg. 2 with
 * M = D/omega + L, Sec. 3.2-3.3).  `visit` numbers the calls of level l
 * within one update (W-cycles visit coarse levels several times). */
static void smooth(ora_problem* p, workspace* ws, int l, int dir, int sigma, uint32_t visit,
                   uint32_t chain, uint32_t m, double* theta, const double* f) {
  level* lv = &p->lv[l];
  int64_t N = lv->N;
  double* g = ws->g;
  for (int64_t i = 0; i < N; ++i) g[i] = f ? f[i] : 0.0;
  uint32_t sweep_word = (visit << 16) | ((uint32_t)l << 8) | ((uint32_t)sigma << 4);
  if (p->beta > 0) {
    for (int j = 0; j < p->beta; ++j) {
      double zeta = draw(p, chain, m, sweep_word, (uint32_t)(j >> 1), j & 1, 1);
      double xi = zeta / sqrt(p->gamma[j]);
      for (int64_t e = lv->BT.ptr[j]; e < lv->BT.ptr[j + 1]; ++e) g[lv->BT.col[e]] += lv->BT.val[e] * xi;
    }
  }
  int nq = p->ncolours;
  double om = p->omega;
  for (int qq = 0; qq < nq; ++qq) {
    int q = dir == 0 ? qq : nq - 1 - qq;
    int c = fwd_colour(p, q);
    for (int64_t t = lv->cstart[q]; t < lv->cstart[q + 1]; ++t) {
      int32_t i = lv->order[t];
      double s = g[i];
      for (int64_t e = lv->A.ptr[i]; e < lv->A.ptr[i + 1]; ++e)
        if (lv->A.col[e] != i) s -= lv->A.val[e] * theta[lv->A.col[e]];
      double z = draw(p, chain, m, sweep_word | (uint32_t)c, lv->pair[i], lv->slot[i], 0);
      if (om == 1.0)
        theta[i] = s / lv->diag[i] + z / sqrt(lv->diag[i]);
      else
        theta[i] = (1.0 - om) * theta[i] + om * (s / lv->diag[i]) + sqrt(om * (2.0 - om) / lv->diag[i]) * z;
    }
  }
  if (p->beta > 0) {
    double* w = ws->w;
    for (int j = 0; j < p->beta; ++j) {
      double acc = 0.0;
      for (int64_t e = lv->BT.ptr[j]; e < lv->BT.ptr[j + 1]; ++e) acc += lv->BT.val[e] * theta[lv->BT.col[e]];
      w[j] = acc;
    }
    const double* G = lv->G[dir];
    for (int64_t r = 0; r < lv->nsupp[dir]; ++r) {
      double acc = 0.0;
      for (int j = 0; j < p->beta; ++j) acc += G[r * p->beta + j] * w[j];
      theta[lv->supp[dir][r]] -= acc;
    }
  }
}

/* Coarsest level (line 3 of Alg. 1).
 * nu0 = 0: exact sample (Sec. 3.5, Cholesky sampler of Sec. 5.1.3):
 *   U^T g = f_0, then U theta_0 = g + z with z ~ N(0, I); the input is ignored.
 * nu0 >= 1: Alg. 5, nu0 symmetric Gibbs sweeps with low-rank correction
 *   (forward then backward Alg. 3, as the paper's experiments use on the
 *   coarsest level, Sec. 5.1.3), starting from the input state. */
static void coarse_sample(ora_problem* p, workspace* ws, uint32_t visit, uint32_t chain, uint32_t m,
                          const double* f, double* theta) {
  if (p->nu0 > 0) {
    for (int j = 0; j < p->nu0; ++j) {
      smooth(p, ws, 0, 0, 2 * j, visit, chain, m, theta, f);
      smooth(p, ws, 0, 1, 2 * j + 1, visit, chain, m, theta, f);
    }
    return;
  }
  int64_t n0 = p->lv[0].N;
  const double* U = p->U;
  double* g = ws->t;
  for (int64_t i = 0; i < n0; ++i) {
    double s = f ? f[i] : 0.0;
    for (int64_t k = 0; k < i; ++k) s -= U[k * n0 + i] * g[k];
    g[i] = s / U[i * n0 + i];
  }
  for (int64_t i = 0; i < n0; ++i) g[i] += draw(p, chain, m, visit << 16, (uint32_t)(i >> 1), (int)(i & 1), 2);
  for (int64_t i = n0 - 1; i >= 0; --i) {
    double s = g[i];
    for (int64_t k = i + 1; k < n0; ++k) s -= U[i * n0 + k] * theta[k];
    theta[i] = s / U[i * n0 + i];
  }
}

/* MGMC_l of Alg. 1.  The finest level calls level L-1 once; every level
 * 1 <= l < L calls level l-1 gamma times (gamma = 1: V-cycle, gamma = 2:
 * W-cycle, as the paper defines them after Alg. 1), the calls after the first
 * starting from the previous coarse state.  ws->visits[l] counts the calls of
 * level l in the current update; the count keys that call's noise. */
static void mgmc_level(ora_problem* p, workspace* ws, int l, uint32_t chain, uint32_t m, double* theta,
                       const double* f) {
  uint32_t visit = ws->visits[l]++;
  if (l == 0) {
    coarse_sample(p, ws, visit, chain, m, f, theta);
    return;
  }
  level* lv = &p->lv[l];
  int64_t N = lv->N;
  for (int j = 0; j < p->nu1; ++j) smooth(p, ws, l, 0, j, visit, chain, m, theta, f);
  /* restriction f_{l-1} = P^T (f_l - At_l theta), At_l = A_l + B_l Gamma^{-1} B_l^T */
  double* r = ws->r;
  for (int64_t i = 0; i < N; ++i) {
    double s = f ? f[i] : 0.0;
    for (int64_t e = lv->A.ptr[i]; e < lv->A.ptr[i + 1]; ++e) s -= lv->A.val[e] * theta[lv->A.col[e]];
    r[i] = s;
  }
  for (int j = 0; j < p->beta; ++j) {
    double acc = 0.0;
    for (int64_t e = lv->BT.ptr[j]; e < lv->BT.ptr[j + 1]; ++e) acc += lv->BT.val[e] * theta[lv->BT.col[e]];
    double v = acc / p->gamma[j];
    for (int64_t e = lv->BT.ptr[j]; e < lv->BT.ptr[j + 1]; ++e) r[lv->BT.col[e]] -= lv->BT.val[e] * v;
  }
  double* fc = ws->f[l - 1];
  double* psi = ws->theta[l - 1];
  int64_t Nc = p->lv[l - 1].N;
  for (int64_t J = 0; J < Nc; ++J) {
    double s = 0.0;
    for (int64_t e = lv->PT.ptr[J]; e < lv->PT.ptr[J + 1]; ++e) s += lv->PT.val[e] * r[lv->PT.col[e]];
    fc[J] = p->restrict_scale * s;
    psi[J] = 0.0;
  }
  int calls = (l == p->L) ? 1 : p->cycle_gamma;
  for (int k = 0; k < calls; ++k) mgmc_level(p, ws, l - 1, chain, m, psi, fc);
  for (int64_t i = 0; i < N; ++i) {
    double s = 0.0;
    for (int64_t e = lv->P.ptr[i]; e < lv->P.ptr[i + 1]; ++e) s += lv->P.val[e] * psi[lv->P.col[e]];
    theta[i] += s;
  }
  for (int j = 0; j < p->nu2; ++j) smooth(p, ws, l, 1, p->nu1 + j, visit, chain, m, theta, f);
}

/* One Markov update: the MGMC cycle, or for the standalone Gibbs sampler of
 * Sec. 5.1.3 nu1 symmetric Gibbs sweeps (forward then backward Alg. 3,
 * i.e. Alg. 4) on the single level. */
static void update(ora_problem* p, workspace* ws, uint32_t chain, uint32_t m, double* theta) {
  for (int l = 0; l <= p->L; ++l) ws->visits[l] = 0;
  if (p->sampler == ORA_SAMPLER_GIBBS) {
    for (int j = 0; j < p->nu1; ++j) {
      smooth(p, ws, p->L, 0, 2 * j, 0, chain, m, theta, p->fL);
      smooth(p, ws, p->L, 1, 2 * j + 1, 0, chain, m, theta, p->fL);
    }
    return;
  }
  mgmc_level(p, ws, p->L, chain, m, theta, p->fL);
}

int ora_cycle(ora_problem* p, int64_t chain, int64_t m, double* theta) {
  workspace ws;
  if (ws_alloc(p, &ws)) { ws_free(&ws, p->L); set_err("allocation failed"); return -1; }
  update(p, &ws, (uint32_t)chain, (uint32_t)m, theta);
  ws_free(&ws, p->L);
  return 0;
}

int ora_chain(ora_problem* p, int64_t chain, int64_t m0, int64_t nsamples, double* theta,
              const double* F, double* qoi, double* traj) {
  workspace ws;
  if (ws_alloc(p, &ws)) { ws_free(&ws, p->L); set_err("allocation failed"); return -1; }
  int64_t N = p->lv[p->L].N;
  for (int64_t k = 0; k < nsamples; ++k) {
    update(p, &ws, (uint32_t)chain, (uint32_t)(m0 + k), theta);
    if (F && qoi) {
      double s = 0.0;
      for (int64_t i = 0; i < N; ++i) s += F[i] * theta[i];
      qoi[k] = s;
    }
    if (traj) memcpy(traj + k * N, theta, (size_t)N * sizeof(double));
  }
  ws_free(&ws, p->L);
  return 0;
}

int ora_smooth(ora_problem* p, int level_index, int direction, int sigma, int64_t chain, int64_t m,
               double* theta, const double* f) {
  int lmin = smoothed_coarsest(p) ? 0 : 1;
  if (level_index < lmin || level_index > p->L || (direction != 0 && direction != 1)) {
    set_err("invalid smoother arguments");
    return -1;
  }
  workspace ws;
  if (ws_alloc(p, &ws)) { ws_free(&ws, p->L); return -1; }
  smooth(p, &ws, level_index, direction, sigma, 0u, (uint32_t)chain, (uint32_t)m, theta, f);
  ws_free(&ws, p->L);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Accessors                                                                 */
/* ------------------------------------------------------------------------ */

int ora_levels(const ora_problem* p) { return p->L + 1; }
int ora_level_n(const ora_problem* p, int l) { return (l < 0 || l > p->L) ? -1 : p->lv[l].n; }
int64_t ora_level_sites(const ora_problem* p, int l) { return (l < 0 || l > p->L) ? -1 : p->lv[l].N; }
int ora_beta(const ora_problem* p) { return p->beta; }

int ora_dense(const ora_problem* p, int l, int what, double* out) {
  if (l < 0 || l > p->L) return -1;
  const level* lv = &p->lv[l];
  int64_t N = lv->N;
  switch (what) {
    case 0:
      memset(out, 0, (size_t)(N * N) * sizeof(double));
      for (int64_t r = 0; r < N; ++r)
        for (int64_t e = lv->A.ptr[r]; e < lv->A.ptr[r + 1]; ++e) out[r * N + lv->A.col[e]] += lv->A.val[e];
      return 0;
    case 1: {
      if (l == 0) return -1;
      int64_t Nc = p->lv[l - 1].N;
      memset(out, 0, (size_t)(N * Nc) * sizeof(double));
      for (int64_t r = 0; r < N; ++r)
        for (int64_t e = lv->P.ptr[r]; e < lv->P.ptr[r + 1]; ++e) out[r * Nc + lv->P.col[e]] += lv->P.val[e];
      return 0;
    }
    case 2:
      memset(out, 0, (size_t)(N * p->beta) * sizeof(double));
      for (int64_t r = 0; r < N; ++r)
        for (int64_t e = lv->B.ptr[r]; e < lv->B.ptr[r + 1]; ++e) out[r * p->beta + lv->B.col[e]] += lv->B.val[e];
      return 0;
    case 3:
    case 4: {
      if (l == 0 || p->beta == 0) return -1;
      int dir = what - 3;
      memset(out, 0, (size_t)(N * p->beta) * sizeof(double));
      for (int64_t r = 0; r < lv->nsupp[dir]; ++r)
        for (int j = 0; j < p->beta; ++j) out[(int64_t)lv->supp[dir][r] * p->beta + j] = lv->G[dir][r * p->beta + j];
      return 0;
    }
    case 5:
      if (l != 0) return -1;
      memcpy(out, p->U, (size_t)(N * N) * sizeof(double));
      return 0;
    case 6: {
      double* a = dense_tilde(p, l);
      if (!a) return -1;
      memcpy(out, a, (size_t)(N * N) * sizeof(double));
      free(a);
      return 0;
    }
    case 7:
      for (int64_t r = 0; r < N; ++r) out[r] = lv->colour[r];
      return 0;
    case 8:
      for (int64_t r = 0; r < N; ++r) out[r] = lv->diag[r];
      return 0;
    default:
      return -1;
  }
}
