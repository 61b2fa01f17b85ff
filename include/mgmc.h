/*
 * mgmc.h -- C ABI of the MI355X Multigrid Monte Carlo sampler.
 *
 * The library draws a Markov chain theta^(0), theta^(1), ... whose law
 * converges to the Gaussian N(At^{-1} f, At^{-1}) with precision
 *   At = A + B Gamma^{-1} B^T
 * (Kazashi, Mueller, Scheichl, arXiv 2407.12149: target of Sec. 5.1 eq.
 * target_distribution, posterior covariance eq. post-cov).  Each update is one
 * MGMC V-cycle theta^(m+1) = MGMC_L(At, f_L, theta^(m)) (Alg. 1, gamma = 1)
 * with colour-ordered random Gauss-Seidel smoothing, the Woodbury low-rank
 * correction of Alg. 3 (omega = 1) on every level when observations are
 * given, Galerkin coarse operators (eq. galerkin_triple_product), transfers
 * R = P^T (Sec. 3.1) and an exact Cholesky sample on the coarsest level
 * (Sec. 3.5).
 *
 * A is the finite-difference operator of Sec. 5.1.1 in divergence form,
 *   (A u)_i = s [kappa^2 u_i + h^-2 sum_k a_{i+e_k/2}(u_i - u_{i+e_k})
 *                                     + a_{i-e_k/2}(u_i - u_{i-e_k})],
 * on the n^dim interior nodes of the unit square/cube with u = 0 on the
 * boundary, h = 1/(n+1), s the operator scale (default h^dim).
 *
 * Conventions shared by every call:
 *   * Site vectors are lexicographic over interior nodes, x fastest:
 *     index (i_1-1) + n (i_2-1) + n^2 (i_3-1), 1 <= i_k <= n.
 *   * Chain states are stored chain-major: theta[c * N + i], N = n^dim.
 *   * Noise is counter-based (Philox4x32-10 with Box-Muller, per site, per
 *     sweep, per sample index m), so sample m of chain c depends only on
 *     (seed, chain_offset + c, m, problem): runs can be split at any m.
 *   * Every call after mgmc_setup is asynchronous on the HIP stream given at
 *     setup; device pointers must stay valid until that stream reaches the
 *     work.  mgmc_setup synchronises that stream before returning.
 *   * Errors are reported by return code; mgmc_last_error() gives a
 *     thread-local message for the last failing call of this thread.  On
 *     MGMC_EINVAL nothing has been written.
 *   * One context per host thread; contexts are independent.
 */
#ifndef MGMC_H
#define MGMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mgmc_ctx mgmc_ctx; /* opaque, owned by the library */

typedef enum {
  MGMC_OK = 0,
  MGMC_EINVAL = 1,      /* invalid argument (shape, NULL pointer, sign) */
  MGMC_ENOMEM = 2,      /* host or device allocation failed */
  MGMC_EDEVICE = 3,     /* a HIP call failed; message carries the HIP error */
  MGMC_ENOTSPD = 4,     /* the coarsest matrix At_0 has no Cholesky factor */
  MGMC_EUNSUPPORTED = 5,
  MGMC_ESTATE = 6       /* call not valid in the context's state */
} mgmc_status;

typedef enum {
  MGMC_FP64 = 0, /* sweeps, noise and state in FP64 */
  MGMC_FP32 = 1  /* sweeps, noise and state in FP32; coarsest sample and
                    low-rank terms in FP64 */
} mgmc_precision;

/* Fine operators of Sec. 5.1.1. */
typedef enum {
  MGMC_OP_FD = 0,     /* finite differences in divergence form (above), 5/7-point */
  MGMC_OP_FEM_Q1 = 1, /* 2D, a = 1: lowest-order bilinear finite elements for
                         -Laplace + kappa^2, the Galerkin matrix of the bilinear
                         form times s / h^2 (9-point) */
  MGMC_OP_SSL13 = 2   /* 2D, a = 1: squared shifted Laplace (-Laplace + kappa^2)^2,
                         s [h^-4 (13-point biharmonic difference) + 2 kappa^2 h^-2
                         (5-point -Laplace) + kappa^4] with u = du/dn = 0 on the
                         boundary (ghost nodes mirror the interior); its Galerkin
                         coarse operators are 25-point and every level sweeps in
                         the nine colours (i_1 mod 3) + 3 (i_2 mod 3), ascending */
} mgmc_operator;

/* Samplers of Sec. 5.1.3. */
typedef enum {
  MGMC_SAMPLER_MGMC = 0,    /* Alg. 1 */
  MGMC_SAMPLER_GIBBS = 1,   /* levels == 1: each update is nu1 symmetric Gibbs sweeps
                               (forward then backward Alg. 3, i.e. Alg. 4) */
  MGMC_SAMPLER_CHOLESKY = 2 /* levels == 1: each update is an independent exact
                               sample theta = At^{-1} f + U^{-1} z, At = U^T U by a
                               banded Cholesky factor in lexicographic order */
} mgmc_sampler;

typedef struct {
  int32_t dim;             /* 2 or 3 */
  int32_t n;               /* interior nodes per dimension, n = 2^k - 1 */
  int32_t levels;          /* 1 <= levels <= k; n_{l-1} = (n_l - 1)/2 */
  int32_t nu1, nu2;        /* pre/post sweeps per level, >= 1, nu1 + nu2 <= 16 */
  double kappa2;           /* kappa^2 of the shifted operator */
  double scale;            /* operator scale s; <= 0 selects h^dim */
  const double* face_coef; /* host; NULL means a = 1, else dim concatenated face
                              arrays, array k with n+1 entries along axis k and
                              n along the others, x fastest: entry f along
                              axis k is a at the face between nodes f and f+1 */
  const double* prolong_w; /* host; NULL means multilinear interpolation, else
                              3^dim weights per coarse node J of the finest
                              transfer (weight of fine node 2J + delta, delta in
                              {-1,0,1}^dim, x fastest), coarse nodes
                              lexicographic; coarser transfers stay multilinear */
  int32_t precision;       /* mgmc_precision */
  int32_t nchains;         /* >= 1 chains sharing the operator */
  int64_t chain_offset;    /* chain c draws the noise of chain id chain_offset + c */
  uint64_t seed;           /* the low 32 bits key the noise */
  /* Fields below default to the plain method when zero. */
  int32_t op;              /* mgmc_operator (MGMC_OP_FD when 0) */
  int32_t cycle_gamma;     /* calls of level l-1 made by every level 1 <= l < L
                              (Alg. 1, gamma_l; the finest level calls once):
                              0 or 1 V-cycle, 2 W-cycle, at most 3 */
  double omega;            /* SOR relaxation of every Gibbs sweep (Sec. 3.3 eq.
                              SOR_smoother, Sec. 3.4 eq. M_lowrank_gibbs),
                              0 < omega < 2; 0 selects 1 */
  int32_t nu0;             /* 0: exact Cholesky sample on level 0; 1..8: Alg. 5,
                              nu0 symmetric Gibbs sweeps with low-rank correction
                              on level 0 (what the paper's experiments run) */
  int32_t sampler;         /* mgmc_sampler (MGMC_SAMPLER_MGMC when 0) */
} mgmc_problem;

typedef struct {
  int32_t beta;            /* number of observations, 1 <= beta <= 2048 */
  const int64_t* ptr;      /* host, beta + 1 offsets into idx/val (CSR over observations) */
  const int32_t* idx;      /* host, fine site index of each weight */
  const double* val;       /* host, weights: column j of B_L (Sec. 2.3 eq. B_ell_definition) */
  const double* gamma;     /* host, beta noise variances sigma_j^2 > 0 (Gamma diagonal) */
} mgmc_obs;

/* Build the hierarchy on the device: fine operator, Galerkin coarse operators
 * A_{l-1} = P^T A_l P and B_{l-1} = P^T B_l (eq. A_ell_1_B_ell_1), the
 * low-rank smoother matrices C = M^{-1} B, S = Gamma + B^T C, G = C S^{-1} for
 * forward and backward sweeps on every level l >= 1 (Alg. 3), and the
 * coarsest Cholesky factor of At_0.  obs = NULL gives the prior (B = 0).
 * hip_stream: a hipStream_t (NULL = default stream) used by every later call.
 * Host arrays are copied; the caller may free them on return.
 * Errors: EINVAL (shape, levels, nu, NULL arrays, gamma <= 0, site index out
 * of range, operator / sampler / gamma / omega / nu0 out of range or not
 * matching dim and levels), ENOTSPD (non-positive diagonal or no Cholesky
 * factor; found on the host before any device work), ENOMEM, EDEVICE,
 * EUNSUPPORTED (some smoothed level whose observation matrix B_l holds more
 * than 8192 - 2 beta weights; a banded factor above 2^31 entries). */
mgmc_status mgmc_setup(const mgmc_problem* problem, const mgmc_obs* obs, void* hip_stream,
                       mgmc_ctx** out);

/* Run updates m0 .. m0+nsamples-1 of every chain for the target with
 * right-hand side f_L = rhs (Alg. 1 with f_L given; rhs = NULL means f = 0,
 * the prior N(0, At^{-1})).
 *   theta: device, [nchains][N] in the context precision, in/out.
 *   rhs:   device FP64 [N] or NULL.
 *   F:     device FP64 [N] weights of the linear quantity of interest
 *          q = F^T theta (Sec. 4 eq. F_matrix), or NULL.
 *   qoi:   device FP64 [nsamples][nchains]: q after each update, or NULL
 *          (both F and qoi, or neither).
 * Errors: EINVAL (NULL theta/ctx, nsamples < 0, m0 < 0, F without qoi). */
mgmc_status mgmc_sample(mgmc_ctx* ctx, int64_t m0, int64_t nsamples, void* theta,
                        const double* rhs, const double* F, double* qoi);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): mgmc_sample with every
 * kernel launched one by one (no graph of its own) and its per-call scratch
 * -- the QoI partial sums and the low-rank vectors t and v -- in a fixed
 * static device array of 4 MiB per GPU instead of the context's buffers.
 * The call allocates nothing; the context (set up by mgmc_setup) still owns
 * the level states, operators and factors.  Every call on one GPU shares that
 * GPU's array (it keeps the last call's contents; nothing in it needs to start
 * at zero), so calls that overlap on one GPU, on any streams, race.
 * Arguments and layout as mgmc_sample.  Errors: as mgmc_sample; EINVAL when
 * the scratch needed, qnb * nchains + 2 beta * nchains doubles (qnb <=
 * max(256, 16384 / nchains)), exceeds 2^19 doubles; EUNSUPPORTED for the
 * Cholesky sampler with a right-hand side (its mean is solved on the host). */
mgmc_status mgmc_sample_noalloc(mgmc_ctx* ctx, int64_t m0, int64_t nsamples, void* theta,
                                const double* rhs, const double* F, double* qoi);

/* As mgmc_sample for the Bayesian posterior: f_L = B_L Gamma^{-1} y
 * (Sec. 2.3 eq. f_ell_definition), recomputed when y changes.
 *   y: host FP64 [beta] observed values.
 * Errors: ESTATE if the context was set up without observations; otherwise
 * as mgmc_sample. */
mgmc_status mgmc_posterior_sample(mgmc_ctx* ctx, const double* y, int64_t m0, int64_t nsamples,
                                  void* theta, const double* F, double* qoi);

/* Number of levels and sites N_l = n_l^dim of level l (0 = coarsest);
 * -1 for an invalid level. */
int32_t mgmc_levels(const mgmc_ctx* ctx);
int64_t mgmc_level_sites(const mgmc_ctx* ctx, int32_t level);

/* Capture one update into a HIP graph and replay it per sample (1) or launch
 * kernels one by one (0, default).  Results are identical either way. */
mgmc_status mgmc_set_graph(mgmc_ctx* ctx, int32_t enabled);

/* Kernel variants; results agree to rounding for every setting (the one-launch
 * 2D sweeps of double-precision contexts draw their normals with a
 * table-driven Box-Muller transform, the other kernels with series).
 *   MGMC_OPT_TILED_SWEEPS: 1 (default) runs each 2D sweep as one launch with
 *     the prolongation fused into the post-smoother; 0 launches one kernel
 *     per colour (the form used for 3D).
 *   MGMC_OPT_SWEEP_VARIANT: form of the one-launch 2D sweep: 0 stages the
 *     stencil through LDS per chain, 1 keeps each thread's stencil in
 *     registers across colours and chains (256 threads per block), 2 the
 *     same with 512 threads per block (taller tiles), 3 (default) chooses
 *     per level, 4 is form 1 with each chain's state tile copied from
 *     memory into LDS by DMA while the previous chain's colour passes run
 *     (5-point levels; 9-point levels take form 1).
 *   MGMC_OPT_CHAINS_PER_BLOCK: chains processed by one block of the 2D
 *     sweep, or (3D contexts) by one thread of the per-site kernels (capped
 *     at 16); 0 (default) chooses from the grid size and precision.
 *   MGMC_OPT_COARSE_FUSED: k >= 1 runs levels 0 .. min(k, m) as one launch
 *     with one workgroup per chain and the levels resident in LDS (2D,
 *     one-launch sweeps), where m is the highest level below the finest
 *     with at most 63 nodes per axis whose levels fit in LDS; 0 (default)
 *     launches them level by level.  Negative values: EINVAL.
 *   MGMC_OPT_LOWRANK_MFMA: 1 (default) computes the low-rank product G t of
 *     all chains with FP64 matrix-core instructions (16 chains per tile; used
 *     for beta <= 512), and on 2D levels with one-launch sweeps (beta <= 128)
 *     the sweep kernel also copies its values at the observation sites, so
 *     that B^T theta, the noise xi and the product take one launch; 2 uses the
 *     matrix cores with a separate launch for B^T theta and xi; 0 uses
 *     vector FMA, 8 chains per pass over G.  Results agree to rounding.
 *   MGMC_OPT_MARCH3D: 1 runs each sweep of a 3D 7-point finest level as one
 *     launch (both parity passes, marching in z over LDS x-y tiles of 64 x 24
 *     sites, out of place), 2 the same with tiles of 64 x 8 sites; 0
 *     (default) as two parity-pass launches.  Results agree to rounding.
 *   MGMC_OPT_RESTRICT3D: 1 (default) forms the residual and its restriction
 *     on 3D 7-point levels in one launch over LDS tiles (the residual stays
 *     on chip); 0 writes the residual to memory and restricts it in a second
 *     launch.  Both sum in the same order.  Values other than 0 and 1:
 *     EINVAL. */
enum {
  MGMC_OPT_TILED_SWEEPS = 1,
  MGMC_OPT_SWEEP_VARIANT = 2,
  MGMC_OPT_CHAINS_PER_BLOCK = 3,
  MGMC_OPT_COARSE_FUSED = 4,
  MGMC_OPT_LOWRANK_MFMA = 5,
  MGMC_OPT_MARCH3D = 6,
  MGMC_OPT_RESTRICT3D = 7
};
mgmc_status mgmc_set_option(mgmc_ctx* ctx, int32_t option, int64_t value);

/* Per-level form of MGMC_OPT_SWEEP_VARIANT or MGMC_OPT_CHAINS_PER_BLOCK for
 * level `level` (0 = coarsest); -1 returns the level to the context-wide
 * setting.  Results agree to rounding for every setting.  Errors: EINVAL. */
mgmc_status mgmc_set_level_option(mgmc_ctx* ctx, int32_t level, int32_t option, int64_t value);

/* Kernel timing of the finest-level smoother sweeps (the hot loop of the
 * update): when enabled, every launch of a finest-level sweep kernel is
 * bracketed by a pair of HIP events on the context stream, in the
 * one-by-one launch mode only.  mgmc_profile_read synchronises the stream
 * and returns the summed kernel time in milliseconds and the number of
 * launches timed since profiling was enabled. */
mgmc_status mgmc_set_profiling(mgmc_ctx* ctx, int32_t enabled);
mgmc_status mgmc_profile_read(mgmc_ctx* ctx, double* total_ms, int64_t* launches);

/* Time nupdates MGMC updates of the context's internal chain states with the
 * current options (graph off), using the right-hand side of the last run; the
 * caller's states are not touched.  Used by the autotuner.  Synchronises. */
mgmc_status mgmc_time_updates(mgmc_ctx* ctx, int32_t nupdates, double* ms);

/* Batches: independent contexts (any sizes, dimensions and precisions) whose
 * updates run as parallel branches of one HIP graph, launched once per group
 * of `updates_per_launch` steps on the batch stream.  The contexts must stay
 * alive while the batch exists and must not be used concurrently. */
typedef struct mgmc_batch mgmc_batch;
mgmc_status mgmc_batch_create(mgmc_ctx* const* ctxs, int32_t count, int32_t updates_per_launch,
                              void* hip_stream, mgmc_batch** out);
/* Updates m0 .. m0+nsamples-1 of every context.  thetas[i], Fs[i], qois[i]
 * follow mgmc_sample for context i (Fs/qois may be NULL, or hold NULLs).
 * Contexts set up with observations sample their posterior for the last y
 * given to mgmc_posterior_sample (ESTATE if none was given), the others the
 * prior. */
mgmc_status mgmc_batch_sample(mgmc_batch* batch, int64_t m0, int64_t nsamples, void* const* thetas,
                              const double* const* Fs, double* const* qois);
mgmc_status mgmc_batch_destroy(mgmc_batch* batch);

/* Learned prolongation.  The sampler keeps its target for any full-rank P
 * with Galerkin coarse operators (invariance theorem of Sec. 4.2, proved for
 * general transfers; Sec. 3.1 notes P is not unique), so the finest transfer
 * may be chosen to speed up mixing.  This network maps the coefficient near
 * each coarse node J to the 9 weights of J in problem.prolong_w (2D):
 *   features: log a on the 24 faces around fine nodes 2J + {-1,0,1}^2;
 *   conv3x3 24->16, ReLU, conv3x3 16->16, ReLU, conv3x3 16->9 (zero padding
 *   on the nc x nc coarse grid, FP32);
 *   rho = softplus(output); weight of J at fine node i = 2J + delta is
 *   rho_J(delta) / sum of rho over the coarse nodes covering i (nodes outside
 *   the grid count 1), and 1 at delta = 0 (FP64).  Equal rho give the
 *   multilinear P.
 * Training minimises the two-grid error reduction of the convergence
 * analysis (Sec. 4.3: error propagator S_post T S_pre with the coarse
 * correction T = I - P (P^T A P)^{-1} P^T A, eq. def-Tell),
 *   L = mean over fields, crops, errors of ||S_b T S_f e||_A^2 / ||e||_A^2,
 * with S_f / S_b one noise-free forward / backward red-black Gauss-Seidel
 * sweep (even coordinate sum first / last), on 15 x 15 coarse-node crops
 * tiling each field (fine window of 31 x 31 nodes with zero Dirichlet data
 * outside it; scale s = h^2).
 * Parameters: pnet_param_count() floats, [W1 16x24x9][b1 16][W2 16x16x9]
 * [b2 16][W3 9x16x9][b3 9], W[cout][cin][t], t = (dx+1) + 3 (dy+1).
 * Calls are asynchronous on hip_stream unless they return host values. */
typedef struct mgmc_pnet mgmc_pnet;
int64_t mgmc_pnet_param_count(void);
/* n: odd fine grid size (nc = (n-1)/2 coarse nodes per axis); buffers for
 * up to max_batch fields and max_errors errors per field; parameters start
 * at 0.  Errors: EINVAL, ENOMEM, EDEVICE. */
mgmc_status mgmc_pnet_create(int32_t n, int32_t max_batch, int32_t max_errors, void* hip_stream,
                             mgmc_pnet** out);
/* host float parameters in/out; set_params also resets the Adam state.
 * Both synchronise. */
mgmc_status mgmc_pnet_set_params(mgmc_pnet* net, const float* params);
mgmc_status mgmc_pnet_get_params(mgmc_pnet* net, float* params);
/* faces: device FP64 [batch][2 (n+1) n] face coefficients (face_coef layout);
 * w: device FP64 [batch][nc*nc][9] learned weights (prolong_w layout). */
mgmc_status mgmc_pnet_weights(mgmc_pnet* net, const double* faces, int32_t batch, double* w);
/* errors: device FP64 [batch][nerrors][n*n] error vectors; kappa2 of the
 * operator.  loss: host FP64 scalar or NULL; grad: host float
 * [param_count] or NULL; synchronises when either is given.  EINVAL when
 * nc < 15 (no crop fits). */
mgmc_status mgmc_pnet_loss_grad(mgmc_pnet* net, const double* faces, const double* errors,
                                int32_t batch, int32_t nerrors, double kappa2, double* loss,
                                float* grad);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on the
 * gradient of the loss; loss (host, may be NULL) receives the loss before the
 * step. */
mgmc_status mgmc_pnet_train_step(mgmc_pnet* net, const double* faces, const double* errors,
                                 int32_t batch, int32_t nerrors, double kappa2, float lr,
                                 double* loss);
mgmc_status mgmc_pnet_destroy(mgmc_pnet* net);

/* Synchronise the context's stream and release everything it owns. */
mgmc_status mgmc_destroy(mgmc_ctx* ctx);

/* Thread-local message of the last failing call ("" if none). */
const char* mgmc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
