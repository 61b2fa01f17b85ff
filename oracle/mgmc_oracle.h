/*
 * mgmc_oracle.h -- plain, slow CPU reference of Multigrid Monte Carlo (MGMC).
 *
 * TEST INFRASTRUCTURE ONLY.  This oracle exists to check the HIP library.
 * Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  The product path never calls it, and it shares no
 * code, header, table or helper with the HIP library.
 *
 * What it computes (Kazashi, Mueller, Scheichl, "Multigrid Monte Carlo
 * Revisited: Theory and Bayesian Inference", arXiv 2407.12149):
 *   * the MGMC Markov update of Alg. 1 (V-cycle, gamma = 1) for the target
 *     N(At^{-1} f, At^{-1}), At = A + B Gamma^{-1} B^T (Sec. 2.3, eq.
 *     post-cov; Sec. 5.1.2 "Posterior");
 *   * random Gibbs smoothing with the low-rank correction of Alg. 3 with
 *     omega = 1 (Sec. 3.4, eqs. M_lowrank_gibbs, lowrank_gibbs_two_steps,
 *     Bellstar_definition), forward before and backward after the coarse
 *     correction (Alg. 4 pairing, Sec. 5.1.3 "Samplers");
 *   * an exact Cholesky sample on the coarsest level (Sec. 3.5 and the
 *     Cholesky-sampler equation of Sec. 5.1.3);
 *   * Galerkin coarse operators A_{l-1} = P^T A_l P, B_{l-1} = P^T B_l
 *     (eqs. A_ell_1_B_ell_1, galerkin_triple_product) with multilinear P
 *     and R = P^T (Sec. 3.1);
 *   * the finite-difference operator s*(kappa^2 u - div(a grad u)) with
 *     homogeneous Dirichlet data on the unit square/cube (Sec. 5.1.1).
 *
 * All arithmetic is FP64, sequential, in the order the paper states the
 * steps.  Sparse matrices are generic CSR; nothing is blocked or fused.
 * Readings where the paper is silent (colour ordering of the Gibbs sweep,
 * operator scale, the Philox counter map) are fixed here and documented with
 * each function.
 */
#ifndef MGMC_ORACLE_H
#define MGMC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ora_problem ora_problem;

/* Philox4x32-10 block function (Salmon, Moraes, Dror, Shaw, SC'11):
 * 10 rounds of the 4x32 Philox S-box with Weyl key schedule. */
void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Two standard normals from one Philox block by the Box-Muller transform:
 * u1 from (x0,x1), u2 from (x2,x3), each the top 53 bits plus one half
 * ulp, scaled by 2^-53 (so 0 < u < 1); out = sqrt(-2 ln u1) (cos, sin)(2 pi u2). */
void ora_normal_pair(const uint32_t ctr[4], const uint32_t key[2], double out[2]);

/* Build the level hierarchy.
 *   dim 2|3, n = 2^k - 1 interior nodes per dimension, h = 1/(n+1),
 *   levels >= 1 (levels == 1: the finest level is sampled by Cholesky),
 *   kappa2 >= 0, scale s (<= 0 selects s = h^dim),
 *   face_coef: NULL (a == 1) or dim concatenated face arrays; array k has
 *     n+1 entries along axis k and n along the others, x fastest,
 *   prolong_w: NULL (multilinear) or 3^dim weights per coarse node of the
 *     finest transfer (offsets delta in {-1,0,1}^dim, x fastest),
 *   nu1, nu2 >= 1 pre/post sweeps, seed (low 32 bits form Philox key word 0).
 * Returns NULL on invalid input (message via ora_last_error). */
ora_problem* ora_create(int dim, int n, int levels, double kappa2, double scale,
                        const double* face_coef, const double* prolong_w,
                        int nu1, int nu2, uint64_t seed);

/* Fine operators (Sec. 5.1.1): finite differences in divergence form (above),
 * lowest-order bilinear finite elements for -Laplace + kappa^2 (2D, a = 1),
 * or the 13-point difference of the squared shifted Laplace
 * (-Laplace + kappa^2)^2 with clamped boundaries (2D, a = 1). */
enum { ORA_OP_FD = 0, ORA_OP_FEM_Q1 = 1, ORA_OP_SSL13 = 2 };
/* Samplers of Sec. 5.1.3: MGMC (Alg. 1), or the standalone Gibbs sampler,
 * nu1 symmetric Gibbs sweeps (Alg. 4) per update on a single level. */
enum { ORA_SAMPLER_MGMC = 0, ORA_SAMPLER_GIBBS = 1 };

/* All set-up choices.  Zero-initialised fields give ora_create's defaults. */
typedef struct {
  int dim, n, levels;
  double kappa2, scale;
  const double* face_coef;
  const double* prolong_w;
  int nu1, nu2;
  uint64_t seed;
  int op;        /* ORA_OP_*; the 13-point operator sweeps in nine colours
                    (i_1 mod 3) + 3 (i_2 mod 3), ascending, on every level */
  int gamma;     /* calls of level l-1 made by levels 1 <= l < L (Alg. 1:
                    1 = V-cycle, 2 = W-cycle; the finest level calls once);
                    0 selects 1 */
  double omega;  /* SOR relaxation of every Gibbs sweep, 0 < omega < 2
                    (Sec. 3.3 eq. SOR_smoother, Sec. 3.4); 0 selects 1 */
  int nu0;       /* 0: exact coarsest sample; 1..8: Alg. 5 with nu0 symmetric
                    Gibbs sweeps with low-rank correction on level 0 */
  int sampler;   /* ORA_SAMPLER_* (Gibbs needs levels == 1) */
} ora_options;
ora_problem* ora_create_ex(const ora_options* options);
void ora_destroy(ora_problem* p);
const char* ora_last_error(void);

/* Observations (Sec. 2.3 eq. B_ell_definition): B_L column j holds the
 * weights val[ptr[j]..ptr[j+1]) at fine sites idx[...]; gamma[j] = sigma_j^2.
 * Precomputes per level and direction C = M^{-1} B, S = Gamma + B^T C and
 * G = C S^{-1} (Alg. 3, setup lines), and the coarsest Cholesky factor.
 * Returns 0 on success. */
int ora_set_obs(ora_problem* p, int beta, const int64_t* ptr, const int32_t* idx,
                const double* val, const double* gamma);

/* Finest right-hand side f_L (NULL: f = 0). */
void ora_set_rhs(ora_problem* p, const double* f);
/* Posterior right-hand side f_L = B_L Gamma^{-1} y (Sec. 2.3, eq. f_ell_definition). */
int ora_set_posterior_rhs(ora_problem* p, const double* y);

/* Noise source.  mode 0: Philox normals (default); 1: every normal is 0;
 * 2: impulse -- the k-th normal drawn (k counted from 0 since the last call
 * of ora_set_noise) is 1, every other is 0.  Used to build the noise-to-state
 * map of one update exactly. */
void ora_set_noise(ora_problem* p, int mode, int64_t impulse_index);
int64_t ora_noise_drawn(const ora_problem* p);

/* Test hook: log every normal drawn, in draw order, as 7 words (key word 0,
 * key word 1, counter words 0..3, slot), into buf (at most cap entries; the
 * count keeps running past cap).  buf = NULL switches logging off.  Used to
 * check that no two draws of a run share a (key, counter, slot), i.e. that
 * the noise components are independent as Alg. 3 requires. */
void ora_set_noise_log(ora_problem* p, uint32_t* buf, int64_t cap);
int64_t ora_noise_log_len(const ora_problem* p);

/* One MGMC update theta <- MGMC_L(At, f_L, theta) for sample index m of chain
 * `chain` (Alg. 1).  theta has N_L entries, lexicographic, x fastest. */
int ora_cycle(ora_problem* p, int64_t chain, int64_t m, double* theta);

/* nsamples consecutive updates m0 .. m0+nsamples-1.  After update m, qoi[k]
 * = F^T theta (if F and qoi non-NULL) and traj[k*N_L ...] = theta (if traj
 * non-NULL), k = m - m0.  Thread-safe in Philox mode for distinct theta. */
int ora_chain(ora_problem* p, int64_t chain, int64_t m0, int64_t nsamples,
              double* theta, const double* F, double* qoi, double* traj);

/* One random smoother application on level `level` (Alg. 3; direction 0 =
 * forward, 1 = backward), sweep index sigma, in place on theta with rhs f. */
int ora_smooth(ora_problem* p, int level, int direction, int sigma, int64_t chain,
               int64_t m, double* theta, const double* f);

/* Test hook for planted-mistake tests: the restriction becomes f_{l-1} =
 * scale * P^T r (the method has scale = 1, R = P^T exactly, Sec. 3.1). */
void ora_set_restriction_scale(ora_problem* p, double scale);

/* Sizes: nodes per dimension and sites of a level (0 = coarsest). */
int ora_levels(const ora_problem* p);
int ora_level_n(const ora_problem* p, int level);
int64_t ora_level_sites(const ora_problem* p, int level);
int ora_beta(const ora_problem* p);

/* Dense copies for tests.  what: 0 prior A_l (N x N), 1 P_l (N_l x N_{l-1}),
 * 2 B_l (N_l x beta), 3 G_fwd (N_l x beta), 4 G_bwd, 5 coarsest Cholesky
 * factor U (upper, At_0 = U^T U), 6 At_l = A_l + B_l Gamma^{-1} B_l^T,
 * 7 colour of each site as double, 8 diagonal A_ii (N).  Returns 0 on
 * success. */
int ora_dense(const ora_problem* p, int level, int what, double* out);

#ifdef __cplusplus
}
#endif
#endif
