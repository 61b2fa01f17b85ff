// C ABI of the MGMC sampler: context set-up, device upload and the V-cycle
// driver (Alg. 1 with gamma = 1, nu1 forward / nu2 backward smoothing steps).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "hierarchy.h"
#include "mgmc.h"
#include "mgmc_internal.h"

namespace {

thread_local std::string g_err;

mgmc_status fail(mgmc_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define MGMC_HIP(expr)                                                                  \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(MGMC_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

inline int64_t host_pidx(const mgmc::Geom& g, const int* i, int dim) {
  return g.o0 + int64_t(i[0] + 3) + int64_t(g.px) * (int64_t(i[1]) + int64_t(g.py) * (dim == 3 ? i[2] : 0));
}

inline int64_t padded_of(const mgmc::Geom& g, int dim, int64_t lin) {
  int i[3] = {0, 0, 0};
  for (int k = 0; k < dim; ++k) {
    i[k] = 1 + int(lin % g.n);
    lin /= g.n;
  }
  return host_pidx(g, i, dim);
}

}  // namespace

// Scratch of mgmc_sample_noalloc: QoI partial sums and the low-rank vectors
// t and v, for callers that cannot allocate.  Each GPU holds its own copy
// until the process ends; host code reaches it only through the address
// hipGetSymbolAddress returns on that device (scratch_ptr).
constexpr int64_t kScratchDoubles = int64_t(1) << 19;  // 4 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (at the first set-up on it).  nullptr on failure.
double* scratch_for_current_device(int* dev_out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  *dev_out = dev;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  return g_scratch_ptr[dev];
}
}  // namespace

namespace mgmc {
int record_error(int status, const char* msg) {
  g_err = msg;
  return status;
}
}  // namespace mgmc

struct mgmc_ctx {
  mgmc_problem prob{};
  hipStream_t stream = nullptr;
  mgmc::Launch L;
  int levels = 0, S = 9, beta = 0, qnb = 0;
  size_t esz = 8;
  std::vector<mgmc::DevLevel> lv;
  double* K = nullptr;
  double* Uinv = nullptr;
  double* gisq = nullptr;  // Gamma^{-1/2}
  double* gam = nullptr;   // Gamma (diagonal)
  double* t = nullptr;     // [nchains][beta] low-rank scratch
  double* v = nullptr;     // [nchains][beta] Gamma^{-1} B^T theta after pre-smoothing
  int64_t* mcur = nullptr;
  double* qpart = nullptr;
  void* fL = nullptr;  // padded finest right-hand side, shared by the chains
  // update forms beyond the tuned V-cycle: W-cycles, SOR relaxation, Alg. 5
  // on level 0 or 5 x 5 stencils run the per-colour kernels level by level
  bool generic = false;
  bool march3d = false;  // one-launch z-marching sweep on the 3D finest level
  int sampler = MGMC_SAMPLER_MGMC, gamma = 1, nu0 = 0;
  // banded single-level exact sampler
  double* Uband = nullptr;
  double* mu = nullptr;     // At^{-1} f of the last right-hand side (null: f = 0)
  double* bandx = nullptr;  // [nchains][N] FP64 scratch of the back substitution
  bool mu_set = false;
  double* scratch = nullptr;  // this device's `scratch` (mgmc_sample_noalloc)
  mgmc::HostHierarchy H;
  std::vector<double> last_y;
  bool posterior_ready = false;
  bool use_graph = false;
  bool tiled = true;    // one launch per 2D sweep; false: one launch per colour
  int sweep_variant = 3;  // 0: LDS-staged tiles, 1/2: segment owners with 256/512 threads, 3: per level
  int sweep_cpb = 0;      // chains per block of the 2D sweeps; 0 picks by size
  std::vector<int> lvl_variant, lvl_cpb;  // per-level overrides, -1 = context-wide setting
  // levels 0..lm run as one workgroup per chain, lm = min(coarse_fused,
  // coarse_lm) (coarse_fused 0: off; coarse_lm 0: not available)
  int coarse_fused = 0;
  int coarse_lm = 0;
  size_t coarse_lds[mgmc::kMaxCoarseLevels] = {};  // LDS bytes per top fused level
  mgmc::CoarseArgs cargs;
  std::vector<void*> allocs;
  // profiling: a ring of event pairs around finest-level sweep launches
  bool profiling = false;
  bool capturing = false;
  std::vector<hipEvent_t> ev_start, ev_stop;
  std::vector<char> ev_pending;
  size_t ev_next = 0;
  double prof_ms = 0.0;
  int64_t prof_launches = 0;

  template <class T>
  mgmc_status alloc(T*& p, size_t count) {
    void* raw = nullptr;
    const size_t bytes = count ? count * sizeof(T) : sizeof(T);
    hipError_t e = hipMalloc(&raw, bytes);
    if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? MGMC_ENOMEM : MGMC_EDEVICE, std::string("hipMalloc: ") + hipGetErrorString(e));
    allocs.push_back(raw);
    p = static_cast<T*>(raw);
    MGMC_HIP(hipMemset(raw, 0, bytes));
    return MGMC_OK;
  }
  mgmc_status alloc_bytes(void*& p, size_t bytes) {
    char* c = nullptr;
    mgmc_status s = alloc(c, bytes);
    p = c;
    return s;
  }
  template <class T>
  mgmc_status upload(T*& p, const std::vector<T>& h) {
    mgmc_status s = alloc(p, h.size());
    if (s != MGMC_OK) return s;
    if (!h.empty()) MGMC_HIP(hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
    return MGMC_OK;
  }
  // Upload a double host vector converted to the context precision.
  mgmc_status upload_real(void*& p, const std::vector<double>& h) {
    if (L.fp32) {
      std::vector<float> f(h.begin(), h.end());
      float* d = nullptr;
      mgmc_status s = upload(d, f);
      p = d;
      return s;
    }
    double* d = nullptr;
    mgmc_status s = upload(d, h);
    p = d;
    return s;
  }
};

namespace {

mgmc_status validate(const mgmc_problem* p, const mgmc_obs* obs) {
  if (!p) return fail(MGMC_EINVAL, "problem is NULL");
  if (p->dim != 2 && p->dim != 3) return fail(MGMC_EINVAL, "dim must be 2 or 3");
  if (p->n < 1 || ((p->n + 1) & p->n) != 0) return fail(MGMC_EINVAL, "n must be 2^k - 1");
  int k = 0;
  while ((1 << k) < p->n + 1) ++k;
  if (p->levels < 1 || p->levels > k) return fail(MGMC_EINVAL, "levels must be in [1, log2(n+1)]");
  if (p->nu1 < 1 || p->nu2 < 1 || p->nu1 + p->nu2 > 16) return fail(MGMC_EINVAL, "nu1, nu2 must be >= 1 with nu1 + nu2 <= 16");
  if (p->nchains < 1 || p->nchains > 65535) return fail(MGMC_EINVAL, "nchains must be in [1, 65535]");
  if (p->precision != MGMC_FP64 && p->precision != MGMC_FP32) return fail(MGMC_EINVAL, "unknown precision");
  if (!(p->kappa2 == p->kappa2) || !(p->scale == p->scale)) return fail(MGMC_EINVAL, "kappa2/scale is NaN");
  if (p->chain_offset < 0 || p->chain_offset + p->nchains > (int64_t(1) << 32)) return fail(MGMC_EINVAL, "chain ids must fit 32 bits");
  const int n0 = ((p->n + 1) >> (p->levels - 1)) - 1;
  int64_t N0 = 1, N = 1;
  for (int d = 0; d < p->dim; ++d) {
    N0 *= n0;
    N *= p->n;
  }
  if (p->op < MGMC_OP_FD || p->op > MGMC_OP_SSL13) return fail(MGMC_EINVAL, "unknown operator");
  if (p->op != MGMC_OP_FD && (p->dim != 2 || p->face_coef))
    return fail(MGMC_EINVAL, "the FEM and squared shifted Laplace operators are 2D with a = 1");
  if (p->cycle_gamma < 0 || p->cycle_gamma > 3) return fail(MGMC_EINVAL, "cycle_gamma must be in [0, 3]");
  if (!(p->omega == 0.0 || (p->omega > 0.0 && p->omega < 2.0))) return fail(MGMC_EINVAL, "omega must lie in (0, 2) (0 selects 1)");
  if (p->nu0 < 0 || p->nu0 > 8) return fail(MGMC_EINVAL, "nu0 must be in [0, 8]");
  if (p->sampler < MGMC_SAMPLER_MGMC || p->sampler > MGMC_SAMPLER_CHOLESKY) return fail(MGMC_EINVAL, "unknown sampler");
  if (p->sampler != MGMC_SAMPLER_MGMC && p->levels != 1) return fail(MGMC_EINVAL, "the Gibbs and Cholesky samplers take levels = 1");
  if (p->sampler == MGMC_SAMPLER_GIBBS && p->nu1 > 8) return fail(MGMC_EINVAL, "the Gibbs sampler takes nu1 <= 8");
  const bool exact_dense = p->sampler == MGMC_SAMPLER_MGMC && p->nu0 == 0;
  if (exact_dense && N0 > 4096) return fail(MGMC_EINVAL, "coarsest level has more than 4096 sites; use more levels");
  if (N > (int64_t(1) << 31) - 1) return fail(MGMC_EINVAL, "grid too large");
  if (p->face_coef) {
    int64_t per = p->n + 1;
    for (int d = 1; d < p->dim; ++d) per *= p->n;
    for (int64_t e = 0; e < per * p->dim; ++e)
      if (!(p->face_coef[e] > 0.0) || !std::isfinite(p->face_coef[e])) return fail(MGMC_EINVAL, "face coefficients must be positive and finite");
  }
  if (p->prolong_w) {
    if (p->levels < 2) return fail(MGMC_EINVAL, "prolong_w needs at least two levels");
    const int nc = (p->n - 1) / 2;
    int64_t cnt = p->dim == 2 ? 9 : 27;
    for (int d = 0; d < p->dim; ++d) cnt *= nc;
    for (int64_t e = 0; e < cnt; ++e)
      if (!std::isfinite(p->prolong_w[e]))
        return fail(MGMC_EINVAL, "prolongation weights must be finite");
  }
  if (obs) {
    if (obs->beta < 1 || obs->beta > 2048) return fail(MGMC_EINVAL, "beta must be in [1, 2048]");
    if (!obs->ptr || !obs->idx || !obs->val || !obs->gamma) return fail(MGMC_EINVAL, "observation arrays must not be NULL");
    if (obs->ptr[0] != 0) return fail(MGMC_EINVAL, "obs ptr[0] must be 0");
    for (int j = 0; j < obs->beta; ++j) {
      if (obs->ptr[j + 1] < obs->ptr[j]) return fail(MGMC_EINVAL, "obs ptr must be non-decreasing");
      if (!(obs->gamma[j] > 0.0) || !std::isfinite(obs->gamma[j])) return fail(MGMC_EINVAL, "gamma must be positive and finite");
      for (int64_t e = obs->ptr[j]; e < obs->ptr[j + 1]; ++e) {
        if (obs->idx[e] < 0 || obs->idx[e] >= N) return fail(MGMC_EINVAL, "observation site out of range");
        if (!std::isfinite(obs->val[e])) return fail(MGMC_EINVAL, "observation weight is NaN");
      }
    }
  }
  return MGMC_OK;
}

mgmc_status upload_level(mgmc_ctx* c, int l) {
  const mgmc::HostHierarchy& H = c->H;
  const mgmc::HostLevel& h = H.lv[l];
  mgmc::DevLevel& d = c->lv[l];
  const int dim = H.dim, S = H.S, nch = c->prob.nchains;
  d.g = mgmc::make_geom(dim, h.n, H.R == 2 ? 2 : 1);
  d.N = h.N;
  d.cross = (l == H.L) && H.op == MGMC_OP_FD;
  const int64_t Np = d.g.Np;
  std::vector<int64_t> pad(h.N);
  for (int64_t i = 0; i < h.N; ++i) pad[i] = padded_of(d.g, dim, i);
  {
    std::vector<double> coef(size_t(S) * Np, 0.0), invd(Np, 0.0), isqd(Np, 0.0);
    const int centre = (S - 1) / 2;
    for (int t = 0; t < S; ++t)
      for (int64_t i = 0; i < h.N; ++i) coef[size_t(t) * Np + pad[i]] = h.st[size_t(t) * h.N + i];
    for (int64_t i = 0; i < h.N; ++i) {
      const double a = h.st[size_t(centre) * h.N + i];
      invd[pad[i]] = 1.0 / a;
      isqd[pad[i]] = 1.0 / std::sqrt(a);
    }
    mgmc_status s;
    if ((s = c->upload_real(d.coef, coef)) != MGMC_OK) return s;
    if ((s = c->upload_real(d.invd, invd)) != MGMC_OK) return s;
    if ((s = c->upload_real(d.isqd, isqd)) != MGMC_OK) return s;
  }
  if (!h.wP.empty()) {
    const mgmc::HostLevel& hc = H.lv[l - 1];
    const mgmc::Geom gc = mgmc::make_geom(dim, hc.n, H.R == 2 ? 2 : 1);
    const int SP = dim == 2 ? 9 : 27;  // prolongation offsets {-1,0,1}^dim
    std::vector<double> w(size_t(SP) * gc.Np, 0.0);
    for (int64_t J = 0; J < hc.N; ++J) {
      const int64_t pj = padded_of(gc, dim, J);
      for (int t = 0; t < SP; ++t) w[size_t(t) * gc.Np + pj] = h.wP[size_t(J) * SP + t];
    }
    mgmc_status s = c->upload(d.wP, w);
    if (s != MGMC_OK) return s;
  }
  mgmc_status s = c->alloc_bytes(d.buf[0], size_t(nch) * Np * c->esz);
  if (s != MGMC_OK) return s;
  const bool smoothed = l >= 1 || H.level0_lowrank;  // level runs smoother sweeps
  if (smoothed) {  // second buffer: out-of-place 2D sweeps, residual scratch
    s = c->alloc_bytes(d.buf[1], size_t(nch) * Np * c->esz);
    if (s != MGMC_OK) return s;
  }
  // a per-chain right-hand side below the finest level; on a 9-point finest
  // level (FEM) too, where the one-launch 2D sweeps take one per chain
  if (l < H.L || (l == H.L && !d.cross && dim == 2 && (l >= 1 || c->prob.sampler == MGMC_SAMPLER_GIBBS))) {
    s = c->alloc_bytes(d.f, size_t(nch) * Np * c->esz);
    if (s != MGMC_OK) return s;
  }
  if (H.beta > 0) {
    const int beta = H.beta;
    std::vector<int64_t> bptr(beta + 1, 0);
    std::vector<int32_t> bidx;
    std::vector<double> bval;
    std::vector<std::vector<std::pair<int32_t, double>>> rows(h.N);
    for (int j = 0; j < beta; ++j) {
      for (const auto& [site, w] : h.Bcol[j]) {
        bidx.push_back(int32_t(pad[site]));
        bval.push_back(w);
        rows[site].push_back({j, w});
      }
      bptr[j + 1] = int64_t(bidx.size());
    }
    d.bnnz = int64_t(bidx.size());
    if (smoothed && d.bnnz > 8192 - 2 * int64_t(beta))
      return fail(MGMC_EUNSUPPORTED, "observation weights on a level exceed the low-rank kernel's LDS (8192 - 2 beta)");
    if ((s = c->upload(d.bptr, bptr)) != MGMC_OK) return s;
    if ((s = c->upload(d.bidx, bidx)) != MGMC_OK) return s;
    if ((s = c->upload(d.bval, bval)) != MGMC_OK) return s;
    int64_t kmax = 0;
    for (int j = 0; j < beta; ++j) kmax = std::max(kmax, bptr[j + 1] - bptr[j]);
    const int bkp = kmax <= 8 ? 8 : kmax == 9 ? 9 : kmax <= 12 ? 12 : kmax <= 16 ? 16 : kmax <= 32 ? 32 : 0;
    if (c->prob.dim == 2 && smoothed && H.R == 1 && d.bnnz > 0 && bkp > 0) {
      // fixed-width slots per column of B (zero padded)
      d.bkp = bkp;
      d.bslots = int64_t(beta) * bkp;
      std::vector<int32_t> slot(size_t(d.bnnz)), pidx(size_t(beta) * bkp, 0);
      std::vector<double> pval(size_t(beta) * bkp, 0.0);
      for (int j = 0; j < beta; ++j)
        for (int64_t e = bptr[j]; e < bptr[j + 1]; ++e) {
          slot[size_t(e)] = int32_t(int64_t(j) * bkp + (e - bptr[j]));
          pidx[size_t(slot[size_t(e)])] = bidx[size_t(e)];
          pval[size_t(slot[size_t(e)])] = bval[size_t(e)];
        }
      if ((s = c->upload(d.bpidx, pidx)) != MGMC_OK) return s;
      if ((s = c->upload(d.bpval, pval)) != MGMC_OK) return s;
      // slots grouped by the 64 x TY tile holding their site, for each tile
      // height of the 2D sweep forms
      const int tiles_x = (h.n + 63) / 64;
      for (int gi = 0; gi < 3; ++gi) {
        const int ty = mgmc::kSnapTY[d.cross ? 1 : 0][gi];
        const int tiles = tiles_x * ((h.n + ty - 1) / ty);
        std::vector<int32_t> tptr(size_t(tiles) + 1, 0), tent(size_t(d.bnnz));
        std::vector<int32_t> tile_of(size_t(d.bnnz));
        for (int64_t e = 0; e < d.bnnz; ++e) {
          const int x = bidx[e] % d.g.px - 3, y = bidx[e] / d.g.px;
          tile_of[e] = ((y - 1) / ty) * tiles_x + (x - 1) / 64;
          ++tptr[size_t(tile_of[e]) + 1];
        }
        for (int t = 0; t < tiles; ++t) tptr[t + 1] += tptr[t];
        std::vector<int32_t> fill(tptr.begin(), tptr.end() - 1);
        for (int64_t e = 0; e < d.bnnz; ++e) tent[size_t(fill[tile_of[e]]++)] = slot[size_t(e)];
        if ((s = c->upload(d.bt_ptr[gi], tptr)) != MGMC_OK) return s;
        if ((s = c->upload(d.bt_ent[gi], tent)) != MGMC_OK) return s;
      }
      // zeroed by alloc; the padding slots are never written
      if ((s = c->alloc(d.bsnap, size_t(nch) * size_t(d.bslots))) != MGMC_OK) return s;
    }
    std::vector<int32_t> brow, brcol;
    std::vector<int64_t> brptr(1, 0);
    std::vector<double> brval;
    for (int64_t i = 0; i < h.N; ++i) {
      if (rows[i].empty()) continue;
      brow.push_back(int32_t(pad[i]));
      for (const auto& [j, w] : rows[i]) {
        brcol.push_back(j);
        brval.push_back(w);
      }
      brptr.push_back(int64_t(brcol.size()));
    }
    d.nbrows = int32_t(brow.size());
    {
      std::vector<int32_t> row_of(size_t(Np), -1);
      for (size_t r = 0; r < brow.size(); ++r) row_of[size_t(brow[r])] = int32_t(r);
      if ((s = c->upload(d.brow_of, row_of)) != MGMC_OK) return s;
    }
    if ((s = c->upload(d.brow, brow)) != MGMC_OK) return s;
    if ((s = c->upload(d.brptr, brptr)) != MGMC_OK) return s;
    if ((s = c->upload(d.brcol, brcol)) != MGMC_OK) return s;
    if ((s = c->upload(d.brval, brval)) != MGMC_OK) return s;
    if (smoothed) {
      for (int dir = 0; dir < 2; ++dir) {
        const int64_t ns = int64_t(h.supp[dir].size());
        d.nsupp[dir] = int32_t(ns);
        std::vector<int32_t> supp(ns);
        std::vector<double> GT(size_t(beta) * ns);
        for (int64_t r = 0; r < ns; ++r) {
          supp[r] = int32_t(pad[h.supp[dir][r]]);
          for (int j = 0; j < beta; ++j) GT[size_t(j) * ns + r] = h.G[dir][size_t(r) * beta + j];
        }
        if ((s = c->upload(d.supp[dir], supp)) != MGMC_OK) return s;
        if ((s = c->upload(d.GT[dir], GT)) != MGMC_OK) return s;
      }
      std::vector<double> SinvT(size_t(beta) * beta);
      for (int a = 0; a < beta; ++a)
        for (int j = 0; j < beta; ++j) SinvT[size_t(j) * beta + a] = h.Sinv[0][size_t(a) * beta + j];
      if ((s = c->upload(d.SinvT, SinvT)) != MGMC_OK) return s;
    }
  }
  return MGMC_OK;
}

// Collect the elapsed time of ring slot k (blocks until its stop event fired).
mgmc_status drain_slot(mgmc_ctx* c, size_t k) {
  if (!c->ev_pending[k]) return MGMC_OK;
  MGMC_HIP(hipEventSynchronize(c->ev_stop[k]));
  float ms = 0.f;
  MGMC_HIP(hipEventElapsedTime(&ms, c->ev_start[k], c->ev_stop[k]));
  c->prof_ms += ms;
  c->prof_launches += 1;
  c->ev_pending[k] = 0;
  return MGMC_OK;
}

// Launch `body` bracketed by events when profiling the finest level.
template <class F>
mgmc_status timed(mgmc_ctx* c, bool finest, F&& body) {
  const bool on = c->profiling && finest && !c->capturing;
  size_t k = 0;
  if (on) {
    k = c->ev_next;
    c->ev_next = (c->ev_next + 1) % c->ev_start.size();
    mgmc_status s = drain_slot(c, k);
    if (s != MGMC_OK) return s;
    MGMC_HIP(hipEventRecord(c->ev_start[k], c->stream));
  }
  hipError_t e = body();
  if (e != hipSuccess) return fail(MGMC_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
  if (on) {
    MGMC_HIP(hipEventRecord(c->ev_stop[k], c->stream));
    c->ev_pending[k] = 1;
  }
  return MGMC_OK;
}

#define MGMC_LAUNCH(expr)                                                              \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) return fail(MGMC_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// One 2D sweep from theta_in into theta_out in the selected kernel form.
hipError_t sweep2d(mgmc_ctx* c, int l, const void* in, void* out, int zero_in, const void* f,
                   int64_t fcs, uint32_t word, int backward, const mgmc::DevLevel* coarse,
                   const void* psi, bool snap) {
  const mgmc::DevLevel& lv = c->lv[l];
  const int sv = c->lvl_variant[l] >= 0 ? c->lvl_variant[l] : c->sweep_variant;
  if (sv == 0)
    return mgmc::launch_sweep_tiled(c->L, lv, in, out, zero_in, f, fcs, word, backward, coarse, psi,
                                    snap);
  // 512-thread blocks (taller tiles, less redundant halo work) or 256-thread
  // blocks; the automatic choice takes 512 threads for FP64 four-colour
  // sweeps with the fused prolongation (register pressure), else 256
  const bool auto512 = !c->L.fp32 && !lv.cross && coarse != nullptr;
  const int variant = (sv == 2 || (sv == 3 && auto512)) ? 1 : (sv == 4 ? 2 : 0);
  int cpb = c->lvl_cpb[l] >= 0 ? c->lvl_cpb[l] : c->sweep_cpb;
  if (cpb <= 0) {
    // each block reuses its stencil registers for a group of up to 8 chains
    // (reloading the stencil per chain costs more than the state traffic),
    // as long as at least 512 blocks remain to fill the device
    const int nch = c->L.nchains;
    const int tys = lv.cross ? (variant == 1 ? 26 : 12) : (variant == 1 ? 22 : 8);
    const int64_t tiles = int64_t((lv.g.n + 63) / 64) * ((lv.g.n + tys - 1) / tys);
    cpb = std::min(nch, 8);
    while (cpb > 1 && tiles * ((nch + cpb - 1) / cpb) < 512) cpb /= 2;
    const int groups = (nch + cpb - 1) / cpb;
    cpb = (nch + groups - 1) / groups;  // balance the groups
  }
  return mgmc::launch_sweep_seg(c->L, lv, in, out, zero_in, f, fcs, word, backward, coarse, psi,
                                variant, cpb, snap);
}

// Whether the low-rank step of level l runs as one launch fed by the sweep's
// snapshot of B's sites (2D one-launch sweeps, matrix-core product).
bool fused_lowrank(const mgmc_ctx* c, const mgmc::DevLevel& lv) {
  return c->beta > 0 && c->beta <= 128 && c->L.lowrank_mfma == 1 && lv.bsnap != nullptr;
}

// One in-place smoother sweep of level l with the per-colour kernels (all
// colours in forward or backward order), as the update forms beyond the tuned
// V-cycle use them: nine-colour passes on 5 x 5 stencils, parity passes on
// 3D 7-point levels, else one launch per colour.
mgmc_status sweep_in_place(mgmc_ctx* c, int l, void* theta, const void* f, int64_t fcs,
                           uint32_t word, bool backward) {
  const mgmc::Launch& L = c->L;
  mgmc::DevLevel& lv = c->lv[l];
  if (c->H.R == 2) {
    for (int qq = 0; qq < 9; ++qq) {
      const int colour = backward ? 8 - qq : qq;
      MGMC_LAUNCH(mgmc::launch_sweep_wide(L, lv, theta, f, fcs, word, colour));
    }
    return MGMC_OK;
  }
  if (c->prob.dim == 3 && lv.cross) {
    for (int pp = 0; pp < 2; ++pp)
      MGMC_LAUNCH(mgmc::launch_sweep_parity3d(L, lv, theta, f, fcs, word, backward ? 1 - pp : pp));
    return MGMC_OK;
  }
  const int nq = 1 << c->prob.dim;
  for (int qq = 0; qq < nq; ++qq) {
    const int q = backward ? nq - 1 - qq : qq;
    MGMC_LAUNCH(mgmc::launch_sweep_colour(L, lv, theta, f, fcs, word, mgmc::forward_colour(c->prob.dim, 2, q)));
  }
  return MGMC_OK;
}

// MGMC_l of Alg. 1 for the general forms (gamma_l calls of level l-1 from
// every level 1 <= l < L, one from the finest; SOR relaxation; Alg. 5 on
// level 0; 5 x 5 stencils), in place on buffer 0 of every level.  visits[l]
// counts the calls of level l in this update and keys their noise.
mgmc_status generic_level(mgmc_ctx* c, int l, const void* fL, std::vector<int>& visits) {
  const mgmc::Launch& L = c->L;
  const int top = c->levels - 1, beta = c->beta;
  const int visit = visits[l]++;
  mgmc::DevLevel& lv = c->lv[l];
  const void* f = (l == top) ? fL : lv.f;
  const int64_t fcs = (l == top) ? 0 : lv.g.Np;
  void* th = lv.buf[0];
  mgmc_status st;
  if (l == 0 && c->nu0 == 0) {
    MGMC_LAUNCH(mgmc::launch_coarsest(L, lv, f, fcs, th, c->K, c->Uinv, mgmc::noise_word(0, 0, visit)));
    return MGMC_OK;
  }
  if (l == 0) {  // Alg. 5: nu0 symmetric Gibbs sweeps with low-rank correction
    for (int j = 0; j < c->nu0; ++j)
      for (int dir = 0; dir < 2; ++dir) {
        const uint32_t word = mgmc::noise_word(0, 2 * j + dir, visit);
        if ((st = sweep_in_place(c, 0, th, f, fcs, word, dir == 1)) != MGMC_OK) return st;
        if (beta) MGMC_LAUNCH(mgmc::launch_lowrank(L, lv, th, dir, word, beta, c->gisq, c->gam, c->t, nullptr));
      }
    return MGMC_OK;
  }
  const int nu1 = c->prob.nu1, nu2 = c->prob.nu2;
  for (int j = 0; j < nu1; ++j) {
    const uint32_t word = mgmc::noise_word(l, j, visit);
    if ((st = sweep_in_place(c, l, th, f, fcs, word, false)) != MGMC_OK) return st;
    if (beta)
      MGMC_LAUNCH(mgmc::launch_lowrank(L, lv, th, 0, word, beta, c->gisq, c->gam, c->t, j == nu1 - 1 ? c->v : nullptr));
  }
  mgmc::DevLevel& cl = c->lv[l - 1];
  mgmc::LowRankRhs lr;
  if (beta) {
    lr.row_of = cl.brow_of;
    lr.ptr = cl.brptr;
    lr.col = cl.brcol;
    lr.val = cl.brval;
    lr.v = c->v;
    lr.beta = beta;
  }
  if (c->H.R == 2)
    MGMC_LAUNCH(mgmc::launch_restrict_wide(L, lv, th, lv.buf[1], cl, f, fcs, lr));
  else if (c->prob.dim == 3)
    MGMC_LAUNCH(mgmc::launch_restrict_2stage(L, lv, th, lv.buf[1], cl, f, fcs, lr));
  else
    MGMC_LAUNCH(mgmc::launch_restrict(L, lv, th, cl, f, fcs, lr));
  // psi^(0) = 0, then gamma_l calls of MGMC_{l-1} (Alg. 1)
  MGMC_LAUNCH(mgmc::launch_fill_zero(L, cl.buf[0], int64_t(L.nchains) * cl.g.Np));
  const int calls = (l == top) ? 1 : c->gamma;
  for (int k = 0; k < calls; ++k)
    if ((st = generic_level(c, l - 1, fL, visits)) != MGMC_OK) return st;
  MGMC_LAUNCH(mgmc::launch_prolong(L, lv, th, cl, cl.buf[0]));
  for (int j = 0; j < nu2; ++j) {
    const uint32_t word = mgmc::noise_word(l, nu1 + j, visit);
    if ((st = sweep_in_place(c, l, th, f, fcs, word, true)) != MGMC_OK) return st;
    if (beta) MGMC_LAUNCH(mgmc::launch_lowrank(L, lv, th, 1, word, beta, c->gisq, c->gam, c->t, nullptr));
  }
  return MGMC_OK;
}

// One MGMC update of every chain (Alg. 1), enqueued on the context stream.
// cur[l] names the buffer holding the state of level l; a tiled sweep reads
// it and writes the other one.  The finest level ends every update in
// buffer 0 (an odd number of sweeps there ends with an in-place sweep).
mgmc_status enqueue_cycle(mgmc_ctx* c, const void* fL, const double* F, double* qoi, int64_t m0) {
  const mgmc::Launch& L = c->L;
  const int top = c->levels - 1, nq = 1 << c->prob.dim, beta = c->beta;
  const int nch = c->prob.nchains;
  const bool tiled = c->tiled && c->prob.dim == 2;
  const int nu1 = c->prob.nu1, nu2 = c->prob.nu2;
  std::vector<int> cur(c->levels, 0);
  auto state = [&](int l) { return c->lv[l].buf[cur[l]]; };
  auto in_place_sweep = [&](int l, const void* f, int64_t fcs, uint32_t word, bool backward) -> mgmc_status {
    mgmc::DevLevel& lv = c->lv[l];
    if (c->prob.dim == 3 && lv.cross && c->tiled) {
      // 7-point level: the four colours of one parity never couple
      for (int pp = 0; pp < 2; ++pp) {
        const int parity = backward ? 1 - pp : pp;
        mgmc_status st = timed(c, l == top, [&] {
          return mgmc::launch_sweep_parity3d(L, lv, state(l), f, fcs, word, parity);
        });
        if (st != MGMC_OK) return st;
      }
      return MGMC_OK;
    }
    for (int qq = 0; qq < nq; ++qq) {
      const int q = backward ? nq - 1 - qq : qq;
      mgmc_status st = timed(c, l == top, [&] {
        return mgmc::launch_sweep_colour(L, lv, state(l), f, fcs, word, mgmc::forward_colour(c->prob.dim, 2, q));
      });
      if (st != MGMC_OK) return st;
    }
    return MGMC_OK;
  };
  if (c->sampler == MGMC_SAMPLER_CHOLESKY) {
    // exact sample of the single level: theta = mu + U^{-1} z
    MGMC_LAUNCH(mgmc::launch_band_sample(L, c->lv[0], c->Uband, c->H.band, c->mu_set ? c->mu : nullptr,
                                         c->bandx, state(0), 0u));
  } else if (c->sampler == MGMC_SAMPLER_GIBBS) {
    // nu1 symmetric Gibbs sweeps (forward then backward Alg. 3) on level 0
    mgmc::DevLevel& lv = c->lv[0];
    const bool fast = tiled && c->H.R == 1 && L.omega == 1.0;
    // a 9-point level (FEM) sweeps with its per-chain copy of f in the one-launch form
    const bool own = fast && lv.f != nullptr;
    const void* fg = own ? lv.f : fL;
    const int64_t fgs = own ? lv.g.Np : 0;
    for (int j = 0; j < nu1; ++j)
      for (int dir = 0; dir < 2; ++dir) {
        const uint32_t word = mgmc::noise_word(0, 2 * j + dir, 0);
        if (fast) {
          const bool snap = fused_lowrank(c, lv);
          mgmc_status st = timed(c, true, [&] {
            return sweep2d(c, 0, state(0), lv.buf[1 - cur[0]], 0, fg, fgs, word, dir, nullptr, nullptr, snap);
          });
          if (st != MGMC_OK) return st;
          cur[0] ^= 1;
          if (snap) {
            MGMC_LAUNCH(mgmc::launch_lowrank_fused(L, lv, state(0), dir, word, beta, c->gisq, c->gam, nullptr));
            continue;
          }
        } else {
          mgmc_status st = sweep_in_place(c, 0, state(0), fL, 0, word, dir == 1);
          if (st != MGMC_OK) return st;
        }
        if (beta) MGMC_LAUNCH(mgmc::launch_lowrank(L, lv, state(0), dir, word, beta, c->gisq, c->gam, c->t, nullptr));
      }
  } else if (c->generic) {
    std::vector<int> visits(c->levels, 0);
    mgmc_status st = generic_level(c, top, fL, visits);
    if (st != MGMC_OK) return st;
  }
  // the bottom levels in one launch when available (2D, one-launch sweeps)
  const int lm = (tiled && c->coarse_fused > 0) ? std::min(c->coarse_fused, c->coarse_lm) : 0;
  if (c->sampler != MGMC_SAMPLER_MGMC || c->generic) {
    // done above
  } else if (top == 0) {
    MGMC_LAUNCH(mgmc::launch_coarsest(L, c->lv[0], fL, 0, state(0), c->K, c->Uinv));
  } else {
    for (int l = top; l >= std::max(1, lm + 1); --l) {
      mgmc::DevLevel& lv = c->lv[l];
      const bool own = l < top || lv.f != nullptr;  // per-chain right-hand side
      const void* f = own ? lv.f : fL;
      const int64_t fcs = own ? lv.g.Np : 0;
      const bool zero_start = l < top;  // psi^(0) = 0 on coarse levels
      if (zero_start && !tiled) MGMC_LAUNCH(mgmc::launch_fill_zero(L, state(l), int64_t(nch) * lv.g.Np));
      for (int j = 0; j < nu1; ++j) {
        const uint32_t word = mgmc::noise_word(l, j);
        double* v_out = j == nu1 - 1 ? c->v : nullptr;
        if (tiled) {
          const int zin = (zero_start && j == 0) ? 1 : 0;
          const bool snap = fused_lowrank(c, lv);
          mgmc_status st = timed(c, l == top, [&] {
            return sweep2d(c, l, state(l), lv.buf[1 - cur[l]], zin, f, fcs, word, 0, nullptr, nullptr,
                           snap);
          });
          if (st != MGMC_OK) return st;
          cur[l] ^= 1;
          if (snap) {
            MGMC_LAUNCH(mgmc::launch_lowrank_fused(L, lv, state(l), 0, word, beta, c->gisq, c->gam, v_out));
            continue;
          }
        } else if (c->march3d && l == top && lv.cross) {
          mgmc_status st = timed(c, true, [&] {
            return mgmc::launch_sweep3d_march(L, lv, state(l), lv.buf[1 - cur[l]], f, word, 0);
          });
          if (st != MGMC_OK) return st;
          cur[l] ^= 1;
        } else {
          mgmc_status st = in_place_sweep(l, f, fcs, word, false);
          if (st != MGMC_OK) return st;
        }
        if (beta)
          MGMC_LAUNCH(mgmc::launch_lowrank(L, lv, state(l), 0, word, beta, c->gisq, c->gam, c->t, v_out));
      }
      mgmc::LowRankRhs lr;
      if (beta) {
        const mgmc::DevLevel& cl = c->lv[l - 1];
        lr.row_of = cl.brow_of;
        lr.ptr = cl.brptr;
        lr.col = cl.brcol;
        lr.val = cl.brval;
        lr.v = c->v;
        lr.beta = beta;
      }
      if (tiled)
        MGMC_LAUNCH(mgmc::launch_restrict_tiled(L, lv, state(l), c->lv[l - 1], f, fcs, lr));
      else if (c->prob.dim == 3 && c->tiled)
        MGMC_LAUNCH(mgmc::launch_restrict_2stage(L, lv, state(l), lv.buf[1 - cur[l]], c->lv[l - 1], f, fcs, lr));
      else
        MGMC_LAUNCH(mgmc::launch_restrict(L, lv, state(l), c->lv[l - 1], f, fcs, lr));
    }
    if (lm >= 1) {
      mgmc::CoarseArgs a = c->cargs;
      a.lm = lm;
      a.f_top = c->lv[lm].f;
      cur[lm] = 0;
      a.theta_top = state(lm);
      MGMC_LAUNCH(mgmc::launch_coarse_vcycle(L, a, c->coarse_lds[lm]));
    } else {
      MGMC_LAUNCH(mgmc::launch_coarsest(L, c->lv[0], c->lv[0].f, c->lv[0].g.Np, state(0), c->K, c->Uinv));
    }
    for (int l = std::max(1, lm + 1); l <= top; ++l) {
      mgmc::DevLevel& lv = c->lv[l];
      const bool own = l < top || lv.f != nullptr;
      const void* f = own ? lv.f : fL;
      const int64_t fcs = own ? lv.g.Np : 0;
      const void* psi = state(l - 1);
      for (int j = 0; j < nu2; ++j) {
        const uint32_t word = mgmc::noise_word(l, nu1 + j);
        const bool last_in_place = l == top && ((nu1 + nu2) & 1) && j == nu2 - 1;
        if (tiled && !last_in_place) {
          const mgmc::DevLevel* coarse = (j == 0) ? &c->lv[l - 1] : nullptr;
          const bool snap = fused_lowrank(c, lv);
          mgmc_status st = timed(c, l == top, [&] {
            return sweep2d(c, l, state(l), lv.buf[1 - cur[l]], 0, f, fcs, word, 1, coarse,
                           coarse ? psi : nullptr, snap);
          });
          if (st != MGMC_OK) return st;
          cur[l] ^= 1;
          if (snap) {
            MGMC_LAUNCH(mgmc::launch_lowrank_fused(L, lv, state(l), 1, word, beta, c->gisq, c->gam, nullptr));
            continue;
          }
        } else {
          if (j == 0) MGMC_LAUNCH(mgmc::launch_prolong(L, lv, state(l), c->lv[l - 1], psi));
          if (c->march3d && l == top && lv.cross && !last_in_place) {
            mgmc_status st = timed(c, true, [&] {
              return mgmc::launch_sweep3d_march(L, lv, state(l), lv.buf[1 - cur[l]], f, word, 1);
            });
            if (st != MGMC_OK) return st;
            cur[l] ^= 1;
          } else {
            mgmc_status st = in_place_sweep(l, f, fcs, word, true);
            if (st != MGMC_OK) return st;
          }
        }
        if (beta)
          MGMC_LAUNCH(mgmc::launch_lowrank(L, lv, state(l), 1, word, beta, c->gisq, c->gam, c->t, nullptr));
      }
    }
  }
  if (cur[top] != 0) return fail(MGMC_EDEVICE, "internal: finest state left in the second buffer");
  // the QoI reduction also advances the sample index
  if (qoi)
    MGMC_LAUNCH(mgmc::launch_qoi(L, c->lv[top], state(top), F, c->qpart, c->qnb, qoi, m0));
  else
    MGMC_LAUNCH(mgmc::launch_advance_m(c->stream, c->mcur));
  return MGMC_OK;
}

mgmc_status run_samples(mgmc_ctx* c, const void* fL, int64_t m0, int64_t nsamples, void* theta,
                        const double* F, double* qoi) {
  const int top = c->levels - 1;
  MGMC_LAUNCH(mgmc::launch_unpack(c->L, c->lv[top], theta, c->lv[top].buf[0]));
  if (c->lv[top].f != nullptr)  // per-chain copies of the finest right-hand side
    MGMC_LAUNCH(mgmc::launch_broadcast(c->L, c->lv[top], fL, c->lv[top].f));
  MGMC_LAUNCH(mgmc::launch_set_m(c->stream, c->mcur, m0));
  if (c->use_graph && c->stream != nullptr && nsamples > 1) {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    MGMC_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    c->capturing = true;
    mgmc_status s = enqueue_cycle(c, fL, F, qoi, m0);
    c->capturing = false;
    hipError_t e = hipStreamEndCapture(c->stream, &graph);
    if (s != MGMC_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return s;
    }
    if (e != hipSuccess) return fail(MGMC_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return fail(MGMC_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    for (int64_t k = 0; k < nsamples && e == hipSuccess; ++k) e = hipGraphLaunch(exec, c->stream);
    // the launches are enqueued; destroying the executable graph is deferred by the runtime
    hipError_t e2 = hipStreamSynchronize(c->stream);
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(MGMC_EDEVICE, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
    if (e2 != hipSuccess) return fail(MGMC_EDEVICE, std::string("hipStreamSynchronize: ") + hipGetErrorString(e2));
  } else {
    for (int64_t k = 0; k < nsamples; ++k) {
      mgmc_status s = enqueue_cycle(c, fL, F, qoi, m0);
      if (s != MGMC_OK) return s;
    }
  }
  MGMC_LAUNCH(mgmc::launch_pack(c->L, c->lv[top], c->lv[top].buf[0], theta));
  return MGMC_OK;
}

// mu = At^{-1} f with the banded factor, which after set-up lives on the
// device only: copied back for the host solve (an empty result on failure).
std::vector<double> band_solve_device(mgmc_ctx* c, const double* f) {
  mgmc::HostHierarchy& H = c->H;
  const size_t cnt = size_t(H.lv[H.L].N) * size_t(H.band + 1);
  H.Uband.resize(cnt);
  if (hipMemcpy(H.Uband.data(), c->Uband, cnt * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
    std::vector<double>().swap(H.Uband);
    return {};
  }
  std::vector<double> mu = mgmc::band_solve(H, f);
  std::vector<double>().swap(H.Uband);
  return mu;
}

mgmc_status check_run_args(mgmc_ctx* c, int64_t m0, int64_t nsamples, void* theta, const double* F,
                           double* qoi) {
  if (!c) return fail(MGMC_EINVAL, "context is NULL");
  if (!theta) return fail(MGMC_EINVAL, "theta is NULL");
  if (nsamples < 0 || m0 < 0) return fail(MGMC_EINVAL, "m0 and nsamples must be >= 0");
  if (m0 + nsamples > (int64_t(1) << 32)) return fail(MGMC_EINVAL, "sample index exceeds 32 bits");
  if ((F == nullptr) != (qoi == nullptr)) return fail(MGMC_EINVAL, "F and qoi must be given together");
  return MGMC_OK;
}

}  // namespace

extern "C" {

mgmc_status mgmc_setup(const mgmc_problem* problem, const mgmc_obs* obs, void* hip_stream,
                       mgmc_ctx** out) {
  g_err.clear();
  if (!out) return fail(MGMC_EINVAL, "out is NULL");
  *out = nullptr;
  mgmc_status s = validate(problem, obs);
  if (s != MGMC_OK) return s;
  mgmc_ctx* c = new (std::nothrow) mgmc_ctx();
  if (!c) return fail(MGMC_ENOMEM, "host allocation failed");
  c->prob = *problem;
  c->prob.face_coef = nullptr;
  c->prob.prolong_w = nullptr;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->levels = problem->levels;
  c->lvl_variant.assign(size_t(c->levels), -1);
  c->lvl_cpb.assign(size_t(c->levels), -1);
  c->S = problem->dim == 2 ? 9 : 27;
  c->esz = problem->precision == MGMC_FP32 ? 4 : 8;
  c->L.stream = c->stream;
  c->L.dim = problem->dim;
  c->L.fp32 = problem->precision == MGMC_FP32;
  c->L.nchains = problem->nchains;
  c->L.seed = uint32_t(problem->seed);
  c->L.chain0 = uint32_t(problem->chain_offset);
  c->L.lowrank_mfma = 1;
  c->L.omega = problem->omega > 0.0 ? problem->omega : 1.0;
  c->sampler = problem->sampler;
  c->gamma = problem->cycle_gamma > 0 ? problem->cycle_gamma : 1;
  c->nu0 = problem->sampler == MGMC_SAMPLER_MGMC ? problem->nu0 : 0;
  c->generic = problem->sampler == MGMC_SAMPLER_MGMC &&
               (c->gamma != 1 || c->L.omega != 1.0 || c->nu0 > 0 || problem->op == MGMC_OP_SSL13);
  std::string err;
  s = mgmc::build_hierarchy(*problem, obs, c->H, err);
  if (s != MGMC_OK) {
    delete c;
    return fail(s, err);
  }
  // the host hierarchy (and its ENOTSPD checks) needs no device
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    delete c;
    return fail(MGMC_EDEVICE, "no HIP device available");
  }
  c->beta = c->H.beta;
  {
    int dev = -1;
    c->scratch = scratch_for_current_device(&dev);
    if (c->scratch == nullptr) {
      delete c;
      return fail(MGMC_EDEVICE, "hipGetSymbolAddress of the no-allocation scratch failed");
    }
  }
  c->lv.assign(c->levels, mgmc::DevLevel{});
  auto cleanup = [&](mgmc_status st) {
    mgmc_destroy(c);
    return st;
  };
  for (int l = 0; l < c->levels; ++l)
    if ((s = upload_level(c, l)) != MGMC_OK) return cleanup(s);
  if (!c->H.K.empty()) {
    if ((s = c->upload(c->K, c->H.K)) != MGMC_OK) return cleanup(s);
    if ((s = c->upload(c->Uinv, c->H.Uinv)) != MGMC_OK) return cleanup(s);
  }
  if (c->sampler == MGMC_SAMPLER_CHOLESKY) {
    if ((s = c->upload(c->Uband, c->H.Uband)) != MGMC_OK) return cleanup(s);
    std::vector<double>().swap(c->H.Uband);
    if ((s = c->alloc(c->mu, size_t(c->lv[0].N))) != MGMC_OK) return cleanup(s);
    if ((s = c->alloc(c->bandx, size_t(c->lv[0].N) * problem->nchains)) != MGMC_OK) return cleanup(s);
  }
  if ((s = c->alloc(c->mcur, 1)) != MGMC_OK) return cleanup(s);
  c->L.mcur = c->mcur;
  {
    std::vector<double> tab(mgmc::kBmTable);
    mgmc::fill_bm_table(tab.data());
    double* d = nullptr;
    if ((s = c->upload(d, tab)) != MGMC_OK) return cleanup(s);
    c->L.bm_table = d;
  }
  const int top = c->levels - 1;
  // QoI partial sums: about 1024 sites per block, at most 16384 partials
  // for the final reduction (one block)
  c->qnb = int(std::min<int64_t>(std::max<int64_t>(256, 16384 / problem->nchains), (c->lv[top].N + 1023) / 1024));
  if (c->qnb < 1) c->qnb = 1;
  if ((s = c->alloc(c->qpart, size_t(c->qnb) * problem->nchains)) != MGMC_OK) return cleanup(s);
  if ((s = c->alloc_bytes(c->fL, size_t(c->lv[top].g.Np) * c->esz)) != MGMC_OK) return cleanup(s);
  if (c->beta > 0) {
    std::vector<double> gisq(c->beta);
    for (int j = 0; j < c->beta; ++j) gisq[j] = 1.0 / std::sqrt(c->H.gamma[j]);
    if ((s = c->upload(c->gisq, gisq)) != MGMC_OK) return cleanup(s);
    if ((s = c->upload(c->gam, c->H.gamma)) != MGMC_OK) return cleanup(s);
    const size_t bc = size_t(c->beta) * problem->nchains;
    if ((s = c->alloc(c->t, bc)) != MGMC_OK) return cleanup(s);
    if ((s = c->alloc(c->v, bc)) != MGMC_OK) return cleanup(s);
  }
  // the bottom of the V-cycle as one launch: the highest level below the
  // finest with at most 63 nodes per axis, if its levels fit in LDS
  if (problem->dim == 2 && top >= 2 && !c->generic && c->sampler == MGMC_SAMPLER_MGMC) {
    int lm = 0;
    for (int l = 1; l < top && l < mgmc::kMaxCoarseLevels; ++l)
      if (c->lv[l].g.n <= 63) lm = l;
    mgmc::CoarseArgs& a = c->cargs;
    a.C.beta = c->beta;
    a.C.nu1 = problem->nu1;
    a.C.nu2 = problem->nu2;
    a.C.gisq = c->gisq;
    a.C.gam = c->gam;
    a.C.K = c->K;
    a.C.Uinv = c->Uinv;
    a.C.mcur = c->mcur;
    a.C.seed = c->L.seed;
    a.C.chain0 = c->L.chain0;
    for (int l = 0; l <= lm; ++l) {
      const mgmc::DevLevel& d = c->lv[l];
      mgmc::CoarseLevel& cl = a.L[l];
      cl.g = d.g;
      cl.coef = d.coef;
      cl.invd = d.invd;
      cl.isqd = d.isqd;
      cl.bptr = d.bptr;
      cl.bidx = d.bidx;
      cl.bval = d.bval;
      for (int dir = 0; dir < 2; ++dir) {
        cl.nsupp[dir] = d.nsupp[dir];
        cl.supp[dir] = d.supp[dir];
        cl.GT[dir] = d.GT[dir];
      }
      cl.SinvT = d.SinvT;
      cl.brow_of = d.brow_of;
      cl.brptr = d.brptr;
      cl.brcol = d.brcol;
      cl.brval = d.brval;
    }
    while (lm >= 1) {
      a.lm = lm;
      int64_t max_bnnz = 0;
      for (int l = 1; l <= lm; ++l) max_bnnz = std::max(max_bnnz, c->lv[l].bnnz);
      const size_t bytes = mgmc::coarse_vcycle_lds(a, c->L.fp32 != 0, max_bnnz);
      if (bytes <= 160 * 1024 && mgmc::coarse_vcycle_prepare(c->L.fp32 != 0, bytes) == hipSuccess) break;
      --lm;
    }
    c->coarse_lm = lm;
    for (int k = 1; k <= lm; ++k) {  // LDS of each smaller top level
      a.lm = k;
      int64_t max_bnnz = 0;
      for (int l = 1; l <= k; ++l) max_bnnz = std::max(max_bnnz, c->lv[l].bnnz);
      c->coarse_lds[k] = mgmc::coarse_vcycle_lds(a, c->L.fp32 != 0, max_bnnz);
    }
    a.lm = lm;
    (void)hipGetLastError();
  }
  // keep only what later calls need on the host: the observation columns
  for (int l = 0; l < c->levels; ++l) {
    mgmc::HostLevel& h = c->H.lv[l];
    if (c->sampler != MGMC_SAMPLER_CHOLESKY) std::vector<double>().swap(h.st);
    for (int d = 0; d < 2; ++d) {
      std::vector<double>().swap(h.C[d]);
      std::vector<double>().swap(h.G[d]);
    }
    if (l < top) std::vector<std::vector<std::pair<int64_t, double>>>().swap(h.Bcol);
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
    return cleanup(fail(MGMC_EDEVICE, "synchronisation after set-up failed"));
  *out = c;
  return MGMC_OK;
}

mgmc_status mgmc_sample(mgmc_ctx* c, int64_t m0, int64_t nsamples, void* theta, const double* rhs,
                        const double* F, double* qoi) {
  g_err.clear();
  mgmc_status s = check_run_args(c, m0, nsamples, theta, F, qoi);
  if (s != MGMC_OK) return s;
  const void* fL = nullptr;
  if (rhs) {
    MGMC_LAUNCH(mgmc::launch_unpack_rhs(c->L, c->lv[c->levels - 1], rhs, c->fL));
    fL = c->fL;
  }
  c->posterior_ready = false;
  if (c->sampler == MGMC_SAMPLER_CHOLESKY) {
    c->mu_set = rhs != nullptr;
    if (rhs) {  // mu = At^{-1} f by the banded factor on the host, once per call
      const int64_t N = c->lv[0].N;
      std::vector<double> f(static_cast<size_t>(N));
      MGMC_HIP(hipStreamSynchronize(c->stream));
      MGMC_HIP(hipMemcpy(f.data(), rhs, size_t(N) * sizeof(double), hipMemcpyDeviceToHost));
      std::vector<double> mu = band_solve_device(c, f.data());
      if (mu.empty()) return fail(MGMC_EDEVICE, "copying the banded factor failed");
      MGMC_HIP(hipMemcpy(c->mu, mu.data(), size_t(N) * sizeof(double), hipMemcpyHostToDevice));
    }
  }
  return run_samples(c, fL, m0, nsamples, theta, F, qoi);
}

mgmc_status mgmc_sample_noalloc(mgmc_ctx* c, int64_t m0, int64_t nsamples, void* theta,
                                const double* rhs, const double* F, double* qoi) {
  g_err.clear();
  mgmc_status s = check_run_args(c, m0, nsamples, theta, F, qoi);
  if (s != MGMC_OK) return s;
  if (c->sampler == MGMC_SAMPLER_CHOLESKY && rhs)
    return fail(MGMC_EUNSUPPORTED, "the Cholesky sampler solves for its mean on the host (allocates)");
  const int64_t nch = c->prob.nchains;
  const int64_t need = int64_t(c->qnb) * nch + 2 * int64_t(c->beta) * nch;
  if (need > kScratchDoubles)
    return fail(MGMC_EINVAL, "scratch need " + std::to_string(need) + " doubles exceeds the " +
                                 std::to_string(kScratchDoubles) + " of the no-allocation scratch");
  const void* fL = nullptr;
  if (rhs) {
    MGMC_LAUNCH(mgmc::launch_unpack_rhs(c->L, c->lv[c->levels - 1], rhs, c->fL));
    fL = c->fL;
  }
  c->posterior_ready = false;
  // the kernels read partial sums and t, v through these pointers: point them
  // into the device's scratch for this call (kernels launched one by one, no
  // graph, no profiling events)
  double* saved[3] = {c->qpart, c->t, c->v};
  const bool graph = c->use_graph, prof = c->profiling;
  c->qpart = c->scratch;
  if (c->beta > 0) {
    c->t = c->scratch + int64_t(c->qnb) * nch;
    c->v = c->t + int64_t(c->beta) * nch;
  }
  c->use_graph = false;
  c->profiling = false;
  s = run_samples(c, fL, m0, nsamples, theta, F, qoi);
  c->qpart = saved[0];
  c->t = saved[1];
  c->v = saved[2];
  c->use_graph = graph;
  c->profiling = prof;
  return s;
}

mgmc_status mgmc_posterior_sample(mgmc_ctx* c, const double* y, int64_t m0, int64_t nsamples,
                                  void* theta, const double* F, double* qoi) {
  g_err.clear();
  mgmc_status s = check_run_args(c, m0, nsamples, theta, F, qoi);
  if (s != MGMC_OK) return s;
  if (c->beta == 0) return fail(MGMC_ESTATE, "context was set up without observations");
  if (!y) return fail(MGMC_EINVAL, "y is NULL");
  for (int j = 0; j < c->beta; ++j)
    if (!std::isfinite(y[j])) return fail(MGMC_EINVAL, "y must be finite");
  const bool same = c->posterior_ready && std::equal(c->last_y.begin(), c->last_y.end(), y);
  if (!same) {
    const int top = c->levels - 1;
    std::vector<double> f = mgmc::posterior_rhs(c->H, y);
    const mgmc::Geom& g = c->lv[top].g;
    std::vector<double> padded(g.Np, 0.0);
    for (int64_t i = 0; i < c->lv[top].N; ++i) padded[padded_of(g, c->prob.dim, i)] = f[i];
    MGMC_HIP(hipStreamSynchronize(c->stream));
    if (c->L.fp32) {
      std::vector<float> pf(padded.begin(), padded.end());
      MGMC_HIP(hipMemcpy(c->fL, pf.data(), pf.size() * sizeof(float), hipMemcpyHostToDevice));
    } else {
      MGMC_HIP(hipMemcpy(c->fL, padded.data(), padded.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    if (c->sampler == MGMC_SAMPLER_CHOLESKY) {
      std::vector<double> mu = band_solve_device(c, f.data());
      if (mu.empty()) return fail(MGMC_EDEVICE, "copying the banded factor failed");
      MGMC_HIP(hipMemcpy(c->mu, mu.data(), mu.size() * sizeof(double), hipMemcpyHostToDevice));
      c->mu_set = true;
    }
    c->last_y.assign(y, y + c->beta);
    c->posterior_ready = true;
  }
  return run_samples(c, c->fL, m0, nsamples, theta, F, qoi);
}

int32_t mgmc_levels(const mgmc_ctx* c) { return c ? c->levels : -1; }

int64_t mgmc_level_sites(const mgmc_ctx* c, int32_t level) {
  if (!c || level < 0 || level >= c->levels) return -1;
  return c->lv[level].N;
}

mgmc_status mgmc_set_graph(mgmc_ctx* c, int32_t enabled) {
  if (!c) return fail(MGMC_EINVAL, "context is NULL");
  c->use_graph = enabled != 0;
  return MGMC_OK;
}

mgmc_status mgmc_set_option(mgmc_ctx* c, int32_t option, int64_t value) {
  if (!c) return fail(MGMC_EINVAL, "context is NULL");
  switch (option) {
    case MGMC_OPT_TILED_SWEEPS:
      c->tiled = value != 0;
      return MGMC_OK;
    case MGMC_OPT_SWEEP_VARIANT:
      if (value < 0 || value > 4) return fail(MGMC_EINVAL, "sweep variant must be 0 .. 4");
      c->sweep_variant = int(value);
      return MGMC_OK;
    case MGMC_OPT_CHAINS_PER_BLOCK:
      if (value < 0 || value > 65535) return fail(MGMC_EINVAL, "chains per block out of range");
      c->sweep_cpb = int(value);
      c->L.cpb_force = c->prob.dim == 3 ? int(value) : 0;
      return MGMC_OK;
    case MGMC_OPT_COARSE_FUSED:
      if (value < 0) return fail(MGMC_EINVAL, "MGMC_OPT_COARSE_FUSED must be >= 0");
      c->coarse_fused = int(std::min<int64_t>(value, mgmc::kMaxCoarseLevels));
      return MGMC_OK;
    case MGMC_OPT_LOWRANK_MFMA:
      if (value < 0 || value > 2) return fail(MGMC_EINVAL, "MGMC_OPT_LOWRANK_MFMA takes 0, 1 or 2");
      c->L.lowrank_mfma = int(value);
      return MGMC_OK;
    case MGMC_OPT_MARCH3D:
      if (value < 0 || value > 2) return fail(MGMC_EINVAL, "MGMC_OPT_MARCH3D takes 0, 1 or 2");
      c->march3d = value != 0 && c->prob.dim == 3;
      c->L.march3d = c->march3d ? int(value) : 0;
      return MGMC_OK;
    case MGMC_OPT_RESTRICT3D:
      if (value < 0 || value > 1) return fail(MGMC_EINVAL, "MGMC_OPT_RESTRICT3D takes 0 or 1");
      c->L.restrict3d = int(value);
      return MGMC_OK;
    default:
      return fail(MGMC_EINVAL, "unknown option");
  }
}

mgmc_status mgmc_set_level_option(mgmc_ctx* c, int32_t level, int32_t option, int64_t value) {
  if (!c) return fail(MGMC_EINVAL, "context is NULL");
  if (level < 0 || level >= c->levels) return fail(MGMC_EINVAL, "level out of range");
  switch (option) {
    case MGMC_OPT_SWEEP_VARIANT:
      if (value < -1 || value > 4) return fail(MGMC_EINVAL, "sweep variant must be -1 .. 4");
      c->lvl_variant[level] = int(value);
      return MGMC_OK;
    case MGMC_OPT_CHAINS_PER_BLOCK:
      if (value < -1 || value > 65535) return fail(MGMC_EINVAL, "chains per block out of range");
      c->lvl_cpb[level] = int(value);
      return MGMC_OK;
    default:
      return fail(MGMC_EINVAL, "option has no per-level form");
  }
}

mgmc_status mgmc_set_profiling(mgmc_ctx* c, int32_t enabled) {
  if (!c) return fail(MGMC_EINVAL, "context is NULL");
  if (enabled && c->ev_start.empty()) {
    const size_t ring = 512;
    c->ev_start.resize(ring);
    c->ev_stop.resize(ring);
    c->ev_pending.assign(ring, 0);
    for (size_t k = 0; k < ring; ++k) {
      MGMC_HIP(hipEventCreate(&c->ev_start[k]));
      MGMC_HIP(hipEventCreate(&c->ev_stop[k]));
    }
  }
  if (enabled) {
    for (size_t k = 0; k < c->ev_pending.size(); ++k) c->ev_pending[k] = 0;
    c->prof_ms = 0.0;
    c->prof_launches = 0;
  }
  c->profiling = enabled != 0;
  return MGMC_OK;
}

mgmc_status mgmc_profile_read(mgmc_ctx* c, double* total_ms, int64_t* launches) {
  if (!c || !total_ms || !launches) return fail(MGMC_EINVAL, "NULL argument");
  MGMC_HIP(hipStreamSynchronize(c->stream));
  for (size_t k = 0; k < c->ev_pending.size(); ++k) {
    mgmc_status s = drain_slot(c, k);
    if (s != MGMC_OK) return s;
  }
  *total_ms = c->prof_ms;
  *launches = c->prof_launches;
  return MGMC_OK;
}

mgmc_status mgmc_time_updates(mgmc_ctx* c, int32_t nupdates, double* ms) {
  if (!c || !ms || nupdates < 1) return fail(MGMC_EINVAL, "invalid timing arguments");
  const void* fL = c->posterior_ready ? c->fL : nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  MGMC_HIP(hipEventCreate(&a));
  MGMC_HIP(hipEventCreate(&b));
  MGMC_HIP(hipStreamSynchronize(c->stream));
  mgmc_status s = MGMC_OK;
  hipError_t e = hipEventRecord(a, c->stream);
  for (int k = 0; k < nupdates && s == MGMC_OK && e == hipSuccess; ++k) s = enqueue_cycle(c, fL, nullptr, nullptr, 0);
  if (e == hipSuccess) e = hipEventRecord(b, c->stream);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (s != MGMC_OK) return s;
  if (e != hipSuccess) return fail(MGMC_EDEVICE, std::string("timing: ") + hipGetErrorString(e));
  *ms = t;
  return MGMC_OK;
}

}  // extern "C"

struct mgmc_batch {
  std::vector<mgmc_ctx*> ctx;
  std::vector<hipStream_t> branch;
  hipStream_t stream = nullptr;
  int per_launch = 1;
};

extern "C" {

mgmc_status mgmc_batch_create(mgmc_ctx* const* ctxs, int32_t count, int32_t updates_per_launch,
                              void* hip_stream, mgmc_batch** out) {
  g_err.clear();
  if (!ctxs || !out || count < 1 || updates_per_launch < 1) return fail(MGMC_EINVAL, "invalid batch arguments");
  if (!hip_stream) return fail(MGMC_EINVAL, "a batch needs a non-default stream (graph capture)");
  *out = nullptr;
  mgmc_batch* b = new (std::nothrow) mgmc_batch();
  if (!b) return fail(MGMC_ENOMEM, "host allocation failed");
  b->stream = static_cast<hipStream_t>(hip_stream);
  b->per_launch = updates_per_launch;
  for (int i = 0; i < count; ++i) {
    if (!ctxs[i]) {
      delete b;
      return fail(MGMC_EINVAL, "NULL context in batch");
    }
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) {
        delete b;
        return fail(MGMC_EINVAL, "context listed twice in batch");
      }
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t x : b->branch) (void)hipStreamDestroy(x);
      delete b;
      return fail(MGMC_EDEVICE, "stream creation failed");
    }
    b->ctx.push_back(ctxs[i]);
    b->branch.push_back(st);
  }
  *out = b;
  return MGMC_OK;
}

mgmc_status mgmc_batch_sample(mgmc_batch* b, int64_t m0, int64_t nsamples, void* const* thetas,
                              const double* const* Fs, double* const* qois) {
  g_err.clear();
  if (!b || !thetas) return fail(MGMC_EINVAL, "invalid batch sample arguments");
  const int nb = int(b->ctx.size());
  for (int i = 0; i < nb; ++i) {
    mgmc_status s = check_run_args(b->ctx[i], m0, nsamples, thetas[i], Fs ? Fs[i] : nullptr, qois ? qois[i] : nullptr);
    if (s != MGMC_OK) return s;
    if (b->ctx[i]->beta > 0 && !b->ctx[i]->posterior_ready) return fail(MGMC_ESTATE, "posterior context without data y");
  }
  if (nsamples == 0) return MGMC_OK;
  // every context works on the batch stream, with its branch stream during capture
  std::vector<hipStream_t> saved(nb);
  for (int i = 0; i < nb; ++i) {
    saved[i] = b->ctx[i]->stream;
    MGMC_HIP(hipStreamSynchronize(saved[i]));
  }
  auto use_stream = [&](int i, hipStream_t st) {
    b->ctx[i]->stream = st;
    b->ctx[i]->L.stream = st;
  };
  auto restore = [&]() {
    for (int i = 0; i < nb; ++i) use_stream(i, saved[i]);
  };
  mgmc_status s = MGMC_OK;
  for (int i = 0; i < nb && s == MGMC_OK; ++i) {
    use_stream(i, b->stream);
    mgmc_ctx* c = b->ctx[i];
    const int top = c->levels - 1;
    hipError_t e = mgmc::launch_unpack(c->L, c->lv[top], thetas[i], c->lv[top].buf[0]);
    if (e == hipSuccess && c->lv[top].f != nullptr)
      e = mgmc::launch_broadcast(c->L, c->lv[top], c->posterior_ready ? c->fL : nullptr, c->lv[top].f);
    if (e == hipSuccess) e = mgmc::launch_set_m(c->stream, c->mcur, m0);
    if (e != hipSuccess) s = fail(MGMC_EDEVICE, std::string("batch start: ") + hipGetErrorString(e));
  }
  // capture `per` updates of every context as parallel branches of one graph
  auto capture = [&](int per, hipGraphExec_t* exec) -> mgmc_status {
    hipGraph_t graph = nullptr;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> join(nb, nullptr);
    MGMC_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    for (int i = 0; i < nb; ++i) MGMC_HIP(hipEventCreateWithFlags(&join[i], hipEventDisableTiming));
    mgmc_status st = MGMC_OK;
    hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) e = hipEventRecord(fork, b->stream);
    for (int i = 0; i < nb && e == hipSuccess && st == MGMC_OK; ++i) {
      e = hipStreamWaitEvent(b->branch[i], fork, 0);
      if (e != hipSuccess) break;
      use_stream(i, b->branch[i]);
      b->ctx[i]->capturing = true;
      mgmc_ctx* c = b->ctx[i];
      const void* fL = c->posterior_ready ? c->fL : nullptr;
      for (int k = 0; k < per && st == MGMC_OK; ++k)
        st = enqueue_cycle(c, fL, Fs ? Fs[i] : nullptr, qois ? qois[i] : nullptr, m0);
      c->capturing = false;
      if (st == MGMC_OK) e = hipEventRecord(join[i], b->branch[i]);
      if (e == hipSuccess && st == MGMC_OK) e = hipStreamWaitEvent(b->stream, join[i], 0);
    }
    hipError_t e2 = hipStreamEndCapture(b->stream, &graph);
    for (int i = 0; i < nb; ++i) use_stream(i, b->stream);
    if (st == MGMC_OK && e == hipSuccess && e2 == hipSuccess) e = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipEventDestroy(fork);
    for (hipEvent_t x : join) (void)hipEventDestroy(x);
    if (st != MGMC_OK) return st;
    if (e != hipSuccess) return fail(MGMC_EDEVICE, std::string("batch capture: ") + hipGetErrorString(e));
    if (e2 != hipSuccess) return fail(MGMC_EDEVICE, std::string("batch capture end: ") + hipGetErrorString(e2));
    return MGMC_OK;
  };
  const int64_t per = std::min<int64_t>(b->per_launch, nsamples);
  const int64_t full = nsamples / per, rest = nsamples % per;
  hipGraphExec_t exec = nullptr, exec_rest = nullptr;
  if (s == MGMC_OK) s = capture(int(per), &exec);
  if (s == MGMC_OK && rest) s = capture(int(rest), &exec_rest);
  hipError_t e = hipSuccess;
  for (int64_t k = 0; s == MGMC_OK && k < full && e == hipSuccess; ++k) e = hipGraphLaunch(exec, b->stream);
  if (s == MGMC_OK && rest && e == hipSuccess) e = hipGraphLaunch(exec_rest, b->stream);
  if (s == MGMC_OK && e != hipSuccess) s = fail(MGMC_EDEVICE, std::string("batch launch: ") + hipGetErrorString(e));
  for (int i = 0; i < nb && s == MGMC_OK; ++i) {
    mgmc_ctx* c = b->ctx[i];
    const int top = c->levels - 1;
    hipError_t e3 = mgmc::launch_pack(c->L, c->lv[top], c->lv[top].buf[0], thetas[i]);
    if (e3 != hipSuccess) s = fail(MGMC_EDEVICE, std::string("batch finish: ") + hipGetErrorString(e3));
  }
  hipError_t e4 = hipStreamSynchronize(b->stream);
  if (exec) (void)hipGraphExecDestroy(exec);
  if (exec_rest) (void)hipGraphExecDestroy(exec_rest);
  restore();
  if (s == MGMC_OK && e4 != hipSuccess) s = fail(MGMC_EDEVICE, std::string("batch sync: ") + hipGetErrorString(e4));
  return s;
}

mgmc_status mgmc_batch_destroy(mgmc_batch* b) {
  if (!b) return MGMC_OK;
  mgmc_status s = MGMC_OK;
  if (hipStreamSynchronize(b->stream) != hipSuccess) s = fail(MGMC_EDEVICE, "stream synchronisation failed");
  for (hipStream_t x : b->branch) (void)hipStreamDestroy(x);
  delete b;
  return s;
}

mgmc_status mgmc_destroy(mgmc_ctx* c) {
  if (!c) return MGMC_OK;
  mgmc_status s = MGMC_OK;
  if (hipStreamSynchronize(c->stream) != hipSuccess) s = fail(MGMC_EDEVICE, "stream synchronisation failed in destroy");
  for (size_t k = 0; k < c->ev_start.size(); ++k) {
    (void)hipEventDestroy(c->ev_start[k]);
    (void)hipEventDestroy(c->ev_stop[k]);
  }
  for (void* p : c->allocs) (void)hipFree(p);
  delete c;
  return s;
}

const char* mgmc_last_error(void) { return g_err.c_str(); }

}  // extern "C"
