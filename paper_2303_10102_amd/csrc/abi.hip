// C ABI of the H-MLE library: handles, validation, state machine, orchestration.
// Every call returns hm_status; errors never cross the ABI as exceptions.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "hm_adjoint.h"
#include "hm_build.h"
#include "hm_factor.h"
#include "hm_internal.h"
#include "hm_trace.h"

namespace hm {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
const char* get_error() { return g_err.c_str(); }

void* dev_alloc(const Ctx* c, size_t bytes) {
  bytes = std::max<size_t>(bytes, 8);
  if (c && c->alloc) return c->alloc(c->uctx, bytes);
  void* p = nullptr;
  return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
}
void dev_free(const Ctx* c, void* p) {
  if (!p) return;
  if (c && c->release) c->release(c->uctx, p);
  else (void)hipFree(p);
}

constexpr int NSCAL = 512;

// One likelihood iteration's state.  All device memory is allocated in hm_H_create.
struct HState {
  Sketch* s = nullptr;
  Model* m = nullptr;
  int p = 0;
  int pidx[5] = {0, 0, 0, 0, 0};
  int nreal = 0;
  int realidx[2] = {-1, -1};   // parameter kind (0 kappa, 1 alpha) of each real derivative
  int realpos[5] = {-1, -1, -1, -1, -1};  // free position -> real derivative slot
  double theta[5] = {0, 0, 0, 0, 0};     // theta_full; [4] the second nugget (bivariate model)
  int state = 0;               // 0 empty, 1 built, 2 factored, 3 parameters prepared
  long long gen = 0;           // incremented by every construction
  long long z_gen = -1;        // construction that z = K~^{-1} y belongs to
  bool have_deriv = false;     // K~_j of the real parameters built at theta (hm_build, not the adjoint)
  int precision = 0;           // 0 FP64; 1 mixed: FP32 MFMA panel products where the policy allows
  int kc = 0;
  PanelSet ps;                 // F and the real panel tangents
  double* D = nullptr;
  double* dDr[2] = {nullptr, nullptr};
  FactorCtx f;
  ParamBufs pb[5];
  LevelBufs lb;
  NodeBufs nb;
  AdjBufs adj;
  double* GtG = nullptr;       // G_c^T G_c per node (shared by the scale parameters)
  double* node_t = nullptr;    // per internal node (2kc)^2 scratch
  double* node_s = nullptr;    // per node kc^2 scratch
  double* ytree = nullptr;
  double* z = nullptr;
  double* r = nullptr;
  double* v = nullptr;
  double* d_scal = nullptr;
  double* d_part = nullptr;
  double* h_scal = nullptr;
  int* h_flags = nullptr;      // pinned copy of the model's device flags
  std::vector<void*> allocs;
  size_t dev_bytes = 0;        // device memory held (allocs)
  // multi-column solve buffers (n x solve_w each): right-hand sides, solution, residual, correction
  int solve_w = 0;
  double* sb[4] = {nullptr, nullptr, nullptr, nullptr};
  // per-phase timing (HIP events around each phase's enqueued work) and counters
  struct Phase {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
    hipEvent_t open = nullptr;
    double ms = 0.0;
  } ph[6];
  std::vector<hipEvent_t> ev_free;
  long long builds = 0, deriv_builds = 0, factors = 0, loglik_evals = 0, grad_evals = 0, fisher_evals = 0,
            reverse_sweeps = 0, solve_rhs = 0;
};

enum : int { PH_BUILD = 0, PH_FACTOR = 1, PH_LOGLIK = 2, PH_FISHER = 3, PH_REVERSE = 4, PH_SOLVE = 5, NPH = 6 };

static hipEvent_t ev_get(HState* h) {
  if (!h->ev_free.empty()) {
    hipEvent_t e = h->ev_free.back();
    h->ev_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  return hipEventCreate(&e) == hipSuccess ? e : nullptr;
}
// accumulate the finished pairs of every phase (wait: block until each has finished)
static void phase_drain(HState* h, bool wait) {
  for (auto& p : h->ph) {
    size_t keep = 0;
    for (size_t i = 0; i < p.pending.size(); ++i) {
      auto pr = p.pending[i];
      if (wait) (void)hipEventSynchronize(pr.second);
      float e = 0.0f;
      if (hipEventQuery(pr.second) == hipSuccess && hipEventElapsedTime(&e, pr.first, pr.second) == hipSuccess) {
        p.ms += e;
        h->ev_free.push_back(pr.first);
        h->ev_free.push_back(pr.second);
      } else {
        p.pending[keep++] = pr;
      }
    }
    p.pending.resize(keep);
  }
}
static void phase_begin(HState* h, int ph) {
  auto& p = h->ph[ph];
  if (p.pending.size() >= 64) phase_drain(h, true);
  p.open = ev_get(h);
  if (p.open) (void)hipEventRecord(p.open, h->m->stream);
}
static void phase_end(HState* h, int ph) {
  auto& p = h->ph[ph];
  if (!p.open) return;
  hipEvent_t b = ev_get(h);
  if (b && hipEventRecord(b, h->m->stream) == hipSuccess) {
    p.pending.emplace_back(p.open, b);
  } else {
    h->ev_free.push_back(p.open);
    if (b) h->ev_free.push_back(b);
  }
  p.open = nullptr;
}

static hm_status dalloc(HState* h, double** p, size_t doubles) {
  void* q = dev_alloc(h->m->ctx, std::max<size_t>(doubles, 1) * sizeof(double));
  h->dev_bytes += std::max<size_t>(doubles, 1) * sizeof(double);
  if (!q) {
    set_error("device allocation of " + std::to_string(doubles * 8) + " bytes failed");
    return HM_E_NOMEM;
  }
  h->allocs.push_back(q);
  *p = (double*)q;
  return HM_OK;
}

hm_status check_theta(const Model* m, const double* t) {
  if (!t) {
    set_error("theta is NULL");
    return HM_E_INVAL;
  }
  for (int i = 0; i < nparams(m); ++i)
    if (!std::isfinite(t[i])) {
      set_error("theta has a non-finite entry");
      return HM_E_NONFINITE;
    }
  if (!(t[2] > 0.0) || !(t[3] > 0.0) || (m->nvars == 2 && !(t[4] > 0.0))) {
    set_error(m->nvars == 2 ? "theta must satisfy tau2_1 > 0, sigma2 > 0, tau2_2 > 0"
                            : "theta must satisfy tau2 > 0, sigma2 > 0");
    return HM_E_INVAL;
  }
  if ((!m->op || m->nvars == 2) && (!(t[0] > 0.0) || !(t[1] >= 0.0))) {
    set_error("theta must satisfy kappa > 0, alpha >= 0, tau2 > 0, sigma2 > 0");
    return HM_E_INVAL;
  }
  return HM_OK;
}

__global__ void k_zero_int(int* p) {
  if (threadIdx.x == 0) *p = 0;
}
// device status flags are cleared by a kernel (no memset node in captured work)
static hm_status clear_flags(Model* m) {
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, m->stream, m->d_flags);
  HM_LAUNCH_CHECK();
  return HM_OK;
}

// y_tree[t] = y_grid[perm[t]]  /  y_grid[perm[t]] = y_tree[t]
// (padding rows: 0 in tree order, skipped in grid order)
__global__ void k_permute(const double* in, double* out, const int* perm, int n, int to_tree) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int g = perm[t];
  if (to_tree) out[t] = g >= 0 ? in[g] : 0.0;
  else if (g >= 0) out[g] = in[t];
}
__global__ void k_add(double* y, const double* x, int n) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) y[t] += x[t];
}

// the same for c columns (leading dimensions ldi, ldo)
__global__ void k_permute_cols(const double* in, long ldi, double* out, long ldo, const int* perm, int n, int c,
                               int to_tree) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * c) return;
  const int t = (int)(e % n), j = (int)(e / n);
  const int g = perm[t];
  if (to_tree) out[t + j * ldo] = g >= 0 ? in[g + j * ldi] : 0.0;
  else if (g >= 0) out[g + j * ldo] = in[t + j * ldi];
}

static hm_status permute(Model* m, const double* in, double* out, int to_tree) {
  hipLaunchKernelGGL(k_permute, dim3(ceil_div(m->n, 256)), dim3(256), 0, m->stream, in, out, m->d_perm, m->n,
                     to_tree);
  HM_LAUNCH_CHECK();
  return HM_OK;
}

// z = K~^{-1} y (w columns of ld n, tree order) with refinement steps against the
// FP64 H-matvec residual (one step; two when the solve sweep runs with FP32 panels);
// r, v: n x w scratch.
static hm_status solve_refined_w(HState* h, const double* y, double* z, double* r, double* v, int w) {
  Model* m = h->m;
  const int n = m->n;
  const long cnt = (long)n * w;
  HM_CHECK(hsolve(h->f, y, z, w));
  const int steps = m->mixed ? 2 : 1;
  for (int it = 0; it < steps; ++it) {
    HM_HIP(hipMemcpyAsync(r, y, cnt * sizeof(double), hipMemcpyDeviceToDevice, m->stream));
    HM_CHECK(hmatvec(h->f, h->D, h->ps.F, nullptr, z, w, r, -1.0, 1.0));   // r = y - K~ z (FP64)
    HM_CHECK(hsolve(h->f, r, v, w));
    hipLaunchKernelGGL(k_add, dim3(ceil_div(cnt, 256)), dim3(256), 0, m->stream, z, v, (int)cnt);
    HM_LAUNCH_CHECK();
  }
  return HM_OK;
}
static hm_status solve_refined(HState* h) { return solve_refined_w(h, h->ytree, h->z, h->r, h->v, 1); }

// scalar slots in d_scal
// scalar slots (device d_scal / pinned h_scal): per free parameter (up to 5) quadratic
// forms, leaf and node traces; the two log-determinant parts; five Fisher terms of
// 5 x 5 entries; the reverse sweep's five sums
enum : int { SC_YZ = 1, SC_QUAD = 2, SC_LTR = 8, SC_NTR = 14, SC_LD = 20, SC_FIM = 24, SC_FT = 25, SC_ITER_END = 150,
             SC_ADJ = 160 };

// out[i nb + j] = <A_i, B_j> for up to 5 x 5 operands (the dot kernels take 4 x 4 at once)
static hm_status dots_any(Model* m, const double* const* A, int na, const double* const* B, int nb, long len,
                          double* out, double* part) {
  if (na <= 4 && nb <= 4) return dots(m, A, na, B, nb, len, out, part);
  for (int i = 0; i < na; ++i) {
    HM_CHECK(dots(m, A + i, 1, B, std::min(nb, 4), len, out + i * nb, part));
    if (nb > 4) HM_CHECK(dots(m, A + i, 1, B + 4, nb - 4, len, out + i * nb + 4, part));
  }
  return HM_OK;
}
static hm_status dots_leafT_any(Model* m, const double* const* A, int na, const double* const* B, int nb,
                                double* out, double* part) {
  if (na <= 4 && nb <= 4) return dots_leafT(m, A, na, B, nb, out, part);
  for (int i = 0; i < na; ++i) {
    HM_CHECK(dots_leafT(m, A + i, 1, B, std::min(nb, 4), out + i * nb, part));
    if (nb > 4) HM_CHECK(dots_leafT(m, A + i, 1, B + 4, nb - 4, out + i * nb + 4, part));
  }
  return HM_OK;
}

static hm_status need_deriv(HState* h, const char* who) {
  if (h->nreal > 0 && !h->have_deriv) {
    set_error(std::string(who) + ": the derivative matrices were not built at this theta "
              "(hm_loglik_grad_adjoint builds K~ only); call hm_build first");
    return HM_E_STATE;
  }
  return HM_OK;
}

static hm_status prepare_params(HState* h) {
  if (h->state >= 3) return HM_OK;
  Model* m = h->m;
  const int n = m->n, kc = h->kc, levels = m->levels;
  bool any_real = false;
  for (int q = 0; q < h->p; ++q) any_real |= (h->pb[q].kind <= 1);
  if (any_real && levels >= 2) {
    // t_c = F_c^T G[c, blocks < depth(c)] shared by every real parameter's Xi
    const long ts = (long)kc * (levels - 1) * kc;
    ReduceJob r{h->ps.F, n, cs_block(kc), h->f.G, n, cs_prefix(kc), 2, levels, h->f.nT, ts, sel_all()};
    HM_CHECK(tree_reduce(m, r));
  }
  if (h->GtG) {
    const long s2 = (long)kc * kc;
    ReduceJob g{h->f.G, n, cs_block(kc), h->f.G, n, cs_block(kc), 1, levels, h->GtG, s2, sel_all()};
    HM_CHECK(tree_reduce(m, g));
  }
  for (int q = 0; q < h->p; ++q) HM_CHECK(param_prepare(h->f, h->pb[q], h->theta, h->f.nT, h->GtG));
  HM_CHECK(node_prep(h->f));
  h->state = 3;
  return HM_OK;
}


// ---------------------------------------------------------------------------
// Iteration phases.  *_enqueue only enqueue device work on the model's stream
// (no host synchronisation), so several handles on different streams overlap;
// fetch_scalars queues the copy of the scalar slots and the device flags to
// pinned host memory; the *_collect / sync_check steps synchronise and check.
// ---------------------------------------------------------------------------
static hm_status fetch_scalars(HState* h, int first, int count) {
  Model* m = h->m;
  HM_HIP(hipMemcpyAsync(h->h_scal + first, h->d_scal + first, count * sizeof(double), hipMemcpyDeviceToHost,
                        m->stream));
  HM_HIP(hipMemcpyAsync(h->h_flags, m->d_flags, sizeof(int), hipMemcpyDeviceToHost, m->stream));
  return HM_OK;
}

// after fetch_scalars: wait, then report construction/factorisation failures
static hm_status sync_check(HState* h, bool factored) {
  HM_HIP(hipStreamSynchronize(h->m->stream));
  const int flags = *h->h_flags;
  if (factored && (flags & (DF_NOT_SPD_LEAF | DF_NOT_SPD_NODE))) {
    set_error(std::string("K~ is not positive definite (") +
              ((flags & DF_NOT_SPD_LEAF) ? "leaf Cholesky" : "node determinant") + ")");
    h->state = 1;
    return HM_E_NOT_SPD;
  }
  if (flags & DF_QR_FAIL) {
    set_error("a sketch QR failed during construction (rank-deficient sample)");
    h->state = 1;
    return HM_E_RANK;
  }
  return HM_OK;
}

static hm_status build_enqueue(HState* h, const double* theta_full, bool deriv) {
  h->m->mixed = h->precision;
  HM_CHECK(check_theta(h->m, theta_full));
  Model* m = h->m;
  h->state = 0;
  h->have_deriv = false;
  std::memcpy(h->theta, theta_full, nparams(m) * sizeof(double));
  if (m->nvars == 1) h->theta[4] = h->theta[2];
  HM_CHECK(clear_flags(m));
  const int n = m->n, kc = h->kc;
  const int nr = deriv ? h->nreal : 0;
  phase_begin(h, PH_BUILD);
  for (int l = 1; l <= m->levels; ++l) {
    const double* XR = h->s->d_XR + (size_t)(l - 1) * kc * n;
    HM_CHECK(level_step(m, h->theta, h->ps, l, XR, kc, h->s->d_k, nr, h->realidx, h->lb, h->nb,
                        h->s->kblk.data()));
  }
  HM_CHECK(leaf_pass(m, h->theta, h->ps, nr, h->realidx, h->lb, h->nb, h->D, deriv ? h->dDr : nullptr));
  phase_end(h, PH_BUILD);
  h->builds += 1;
  h->deriv_builds += (deriv && h->nreal > 0) ? 1 : 0;
  h->state = 1;
  h->have_deriv = deriv;
  ++h->gen;
  return HM_OK;
}

static hm_status factor_enqueue(HState* h) {
  h->m->mixed = h->precision;
  Model* m = h->m;
  phase_begin(h, PH_FACTOR);
  HM_CHECK(factorize(h->f));
  // log|K~| = sum of leaf and node parts
  HM_CHECK(sum_scalar(m, h->f.logdet_leaf, m->nleaves, 0, h->d_scal + SC_LD, h->d_part));
  HM_CHECK(sum_scalar(m, h->f.logdet_node, (1 << m->levels) - 1, 0, h->d_scal + SC_LD + 1, h->d_part));
  phase_end(h, PH_FACTOR);
  h->factors += 1;
  h->state = 2;
  return HM_OK;
}

static hm_status loglik_enqueue(HState* h, const double* y, bool want_grad) {
  h->m->mixed = h->precision;
  Model* m = h->m;
  const int n = m->n;
  phase_begin(h, PH_LOGLIK);
  h->loglik_evals += 1;
  HM_CHECK(permute(m, y, h->ytree, 1));
  HM_CHECK(solve_refined(h));
  const double* yv[1] = {h->ytree};
  const double* zv[1] = {h->z};
  HM_CHECK(dots(m, yv, 1, zv, 1, n, h->d_scal + SC_YZ, h->d_part));
  h->z_gen = h->gen;
  if (!want_grad || h->p == 0) {
    phase_end(h, PH_LOGLIK);
    return HM_OK;
  }
  h->grad_evals += 1;
  HM_CHECK(prepare_params(h));
  for (int q = 0; q < h->p; ++q) {
    ParamBufs& pb = h->pb[q];
    // z^T K~_j z
    HM_CHECK(hmatvec(h->f, pb.dD, h->ps.F, pb.dF, h->z, 1, h->v, 1.0, 0.0));
    const double* vv[1] = {h->v};
    HM_CHECK(dots(m, zv, 1, vv, 1, n, h->d_scal + SC_QUAD + q, h->d_part));
    // tr(K~^{-1} K~_j) = sum_L tr(Y_L) - sum_P <N_P, PsiP>
    HM_CHECK(sum_scalar(m, pb.Y, (long)m->nleaves * m->nl, m->nl, h->d_scal + SC_LTR + q, h->d_part));
    HM_CHECK(node_psi(h->f, pb, h->node_s));
  }
  // node part of every trace: <N_P, PsiP^j> summed over internal nodes
  const long ms = 4L * h->kc * h->kc;
  const double* nv[1] = {h->f.Nn};
  const double* pv[5];
  for (int q = 0; q < h->p; ++q) pv[q] = h->pb[q].PsiP;
  HM_CHECK(dots_any(m, nv, 1, pv, h->p, ((1L << m->levels) - 1) * ms, h->d_scal + SC_NTR, h->d_part));
  phase_end(h, PH_LOGLIK);
  return HM_OK;
}

static hm_status loglik_collect(HState* h, double* loglik, double* grad) {
  const int n = h->m->n_real;
  const double logdet = h->h_scal[SC_LD] + h->h_scal[SC_LD + 1];
  const double yz = h->h_scal[SC_YZ];
  *loglik = -0.5 * n * std::log(2.0 * M_PI) - 0.5 * logdet - 0.5 * yz;
  if (!std::isfinite(*loglik)) {
    set_error("non-finite log-likelihood");
    return HM_E_NONFINITE;
  }
  if (grad) {
    for (int q = 0; q < h->p; ++q) {
      const double tr = h->h_scal[SC_LTR + q] - h->h_scal[SC_NTR + q];
      grad[q] = 0.5 * tr - 0.5 * h->h_scal[SC_QUAD + q];
    }
  }
  return HM_OK;
}

static hm_status fisher_enqueue(HState* h) {
  h->m->mixed = h->precision;
  Model* m = h->m;
  const int p = h->p;
  phase_begin(h, PH_FISHER);
  h->fisher_evals += 1;
  HM_CHECK(prepare_params(h));
  // tau2 before sigma2: sigma2's tangent sweep is a combination of tau2's (one nugget)
  int qt = -1;
  for (int q = 0; q < p; ++q)
    if (h->pb[q].kind == 2 && m->nvars == 1) qt = q;
  int order[5], no = 0;
  for (int q = 0; q < p; ++q)
    if (h->pb[q].kind != 3) order[no++] = q;
  for (int q = 0; q < p; ++q)
    if (h->pb[q].kind == 3) order[no++] = q;
  for (int i = 0; i < p; ++i) {
    const int q = order[i];
    if (h->pb[q].kind == 3 && qt >= 0) HM_CHECK(scale_sweep(h->f, h->pb[q], h->pb[qt], h->theta));
    else HM_CHECK(tangent_sweep(h->f, h->pb[q]));
    HM_CHECK(node_psi(h->f, h->pb[q], h->node_s));
    HM_CHECK(node_lam(h->f, h->pb[q], h->node_t, h->node_s));
    HM_CHECK(panel_products(h->f, h->pb[q]));
  }
  const int n = m->n, kc = h->kc, levels = m->levels;
  const long pset = (long)n * levels * kc;
  const long s2 = (long)kc * kc;
  const long nint = (1 << levels) - 1, nodes = (2L << levels) - 1;
  const double *A[5], *B[5];
  double* out = h->d_scal + SC_FIM;
  // term 0: 1/2 sum_L tr(Y^i_L Y^j_L)  (Y^j transposed is dD_j Dinv)
  for (int q = 0; q < p; ++q) { A[q] = h->pb[q].Y; B[q] = h->pb[q].Y; }
  HM_CHECK(dots_leafT_any(m, A, p, B, p, out + 0 * SC_FT, h->d_part));
  // term 1: -1/2 <Lam^i, PsiP^j>
  for (int q = 0; q < p; ++q) { A[q] = h->pb[q].Lam; B[q] = h->pb[q].PsiP; }
  HM_CHECK(dots_any(m, A, p, B, p, nint * 4 * s2, out + 1 * SC_FT, h->d_part));
  // term 2: <Gh^i, Xi^j>
  for (int q = 0; q < p; ++q) { A[q] = h->pb[q].Gh; B[q] = h->pb[q].Xi; }
  HM_CHECK(dots_any(m, A, p, B, p, pset, out + 2 * SC_FT, h->d_part));
  // term 3: <Hh^i, dF^j>
  for (int q = 0; q < p; ++q) { A[q] = h->pb[q].Hh; B[q] = h->pb[q].dF; }
  HM_CHECK(dots_any(m, A, p, B, p, pset, out + 3 * SC_FT, h->d_part));
  // term 4: <Vt^i, E^j> over non-root nodes
  for (int q = 0; q < p; ++q) { A[q] = h->pb[q].Vt + s2; B[q] = h->pb[q].E + s2; }
  HM_CHECK(dots_any(m, A, p, B, p, (nodes - 1) * s2, out + 4 * SC_FT, h->d_part));
  phase_end(h, PH_FISHER);
  return HM_OK;
}

static hm_status fisher_collect(HState* h, double* fim) {
  const int p = h->p;
  const double* t = h->h_scal + SC_FIM;
  for (int i = 0; i < p; ++i)
    for (int j = 0; j < p; ++j) {
      const int q = i * p + j;
      fim[q] = 0.5 * t[q] - 0.5 * t[SC_FT + q] + t[2 * SC_FT + q] + t[3 * SC_FT + q] + t[4 * SC_FT + q];
      if (!std::isfinite(fim[q])) {
        set_error("non-finite Fisher information");
        return HM_E_NONFINITE;
      }
    }
  return HM_OK;
}

// One whole iteration without a host synchronisation (build, factor, L~ and
// gradient, Fisher), ending with the copy of the scalars to pinned memory.
static hm_status iteration_enqueue(HState* h, const double* theta_full, const double* y, bool want_grad,
                                   bool want_fim) {
  HM_CHECK(build_enqueue(h, theta_full, true));
  HM_CHECK(factor_enqueue(h));
  HM_CHECK(loglik_enqueue(h, y, want_grad));
  if (want_fim && h->p > 0) HM_CHECK(fisher_enqueue(h));
  HM_CHECK(fetch_scalars(h, 0, SC_ITER_END));
  return HM_OK;
}

static hm_status iteration_collect(HState* h, double* loglik, double* grad, double* fim) {
  HM_CHECK(sync_check(h, true));
  phase_drain(h, false);
  HM_CHECK(loglik_collect(h, loglik, grad));
  if (fim && h->p > 0) HM_CHECK(fisher_collect(h, fim));
  return HM_OK;
}

}  // namespace hm

using namespace hm;

struct hm_sketch {
  Sketch s;
};
struct hm_H {
  HState h;
};

extern "C" {

const char* hm_last_error(void) { return get_error(); }

struct Rect {
  int x0, y0, w, h;
};
// leaves of the recursive bisection of the N (x N) grid, left to right
static std::vector<Rect> leaf_rects(int dim, int N, int levels) {
  std::vector<Rect> r{{0, 0, N, dim == 2 ? N : 1}};
  for (int d = 0; d < levels; ++d) {
    std::vector<Rect> nx;
    nx.reserve(r.size() * 2);
    for (const Rect& q : r) {
      if (q.w >= q.h) {
        const int wl = q.w / 2;
        nx.push_back({q.x0, q.y0, wl, q.h});
        nx.push_back({q.x0 + wl, q.y0, q.w - wl, q.h});
      } else {
        const int hl = q.h / 2;
        nx.push_back({q.x0, q.y0, q.w, hl});
        nx.push_back({q.x0, q.y0 + hl, q.w, q.h - hl});
      }
    }
    r.swap(nx);
  }
  return r;
}

// Leaves of the KD-tree of a point set (xy: n x dim row-major): a node's points are
// split along the longer side of their bounding box (x on ties), the floor(m/2) with
// the smallest coordinate (ties: the other coordinate, then the index) going left;
// each leaf lists its points in increasing index.
static std::vector<std::vector<int>> point_leaves(int dim, const double* xy, int n, int levels) {
  std::vector<std::vector<int>> nodes(1);
  nodes[0].resize(n);
  for (int i = 0; i < n; ++i) nodes[0][i] = i;
  auto c = [&](int i, int a) { return xy[(size_t)i * dim + a]; };
  for (int d = 0; d < levels; ++d) {
    std::vector<std::vector<int>> nx;
    nx.reserve(nodes.size() * 2);
    for (std::vector<int>& v : nodes) {
      int axis = 0;
      if (dim == 2 && !v.empty()) {
        double x0 = c(v[0], 0), x1 = x0, y0 = c(v[0], 1), y1 = y0;
        for (int i : v) {
          x0 = std::min(x0, c(i, 0));
          x1 = std::max(x1, c(i, 0));
          y0 = std::min(y0, c(i, 1));
          y1 = std::max(y1, c(i, 1));
        }
        axis = (y1 - y0 > x1 - x0) ? 1 : 0;
      }
      const int other = (dim == 2) ? 1 - axis : axis;
      std::sort(v.begin(), v.end(), [&](int a, int b) {
        if (c(a, axis) != c(b, axis)) return c(a, axis) < c(b, axis);
        if (c(a, other) != c(b, other)) return c(a, other) < c(b, other);
        return a < b;
      });
      const size_t half = v.size() / 2;
      nx.emplace_back(v.begin(), v.begin() + half);
      nx.emplace_back(v.begin() + half, v.end());
    }
    nodes.swap(nx);
  }
  for (std::vector<int>& v : nodes) std::sort(v.begin(), v.end());
  return nodes;
}

}  // extern "C"

namespace hm {

// A model on an N (x N) Dirichlet grid with spacing h, its device memory from ctx.
hm_status model_create(Ctx* ctx, int device, void* stream, int dim, int N, double h, int leaf,
                       hm_model** out) {
  if (!out) {
    set_error("out is NULL");
    return HM_E_INVAL;
  }
  *out = nullptr;
  if ((dim != 1 && dim != 2) || N < 2 || leaf < 1) {
    set_error("need dim in {1,2}, N >= 2, leaf >= 1");
    return HM_E_INVAL;
  }
  if (!(h > 0.0) || !std::isfinite(h)) {
    set_error("the grid spacing h must be positive and finite");
    return HM_E_INVAL;
  }
  const long n = (dim == 2) ? (long)N * N : N;
  if (n > (1L << 26)) {
    set_error("grid too large");
    return HM_E_INVAL;
  }
  int levels = (int)std::floor(std::log2((double)n / leaf) + 1e-12);
  if (levels < 1 || levels > 20) {
    set_error("need n >= 2*leaf");
    return HM_E_INVAL;
  }
  // The tree (Sec. 5.2, KD-tree ordering): recursive bisection of the grid rectangle,
  // splitting the longer side (x on ties), the left child taking floor(side / 2) lines.
  // If every split is even the leaves are equal and the tree position has a closed
  // form; otherwise every leaf is stored padded to the largest (see Model).
  std::vector<Rect> leaves = leaf_rects(dim, N, levels);
  bool uniform = true;
  {
    long w = N, hh = (dim == 2) ? N : 1;
    for (int d = 0; d < levels; ++d) {
      long& side = (w >= hh) ? w : hh;
      uniform = uniform && side % 2 == 0;
      side /= 2;
    }
  }
  int nlp = 0, nlmin = (int)n;
  for (const Rect& r : leaves) {
    nlp = std::max(nlp, r.w * r.h);
    nlmin = std::min(nlmin, r.w * r.h);
  }
  if (nlmin < 1) {
    set_error("the tree has an empty leaf: choose a larger leaf size");
    return HM_E_INVAL;
  }
  // the panel reduce reads rows in groups of four inside a leaf: a leaf size that is
  // not a multiple of four is stored padded to the next one
  if (nlp % 4) {
    nlp = (nlp + 3) / 4 * 4;
    uniform = false;
  }
  const long rows = (long)nlp << levels;
  if (rows > (1L << 27)) {
    set_error("grid too large");
    return HM_E_INVAL;
  }
  if (hipSetDevice(device) != hipSuccess) {
    set_error("hipSetDevice failed");
    return HM_E_DEVICE;
  }
  hm_model* hm_ = new hm_model();
  Model* m = &hm_->m;
  m->own_ctx.device = device;
  m->own_ctx.stream = (hipStream_t)stream;
  m->ctx = ctx ? ctx : &m->own_ctx;
  m->device = device;
  m->stream = (hipStream_t)stream;
  m->dim = dim;
  m->N = N;
  m->n = (int)rows;
  m->n_real = (int)n;
  m->uniform = uniform;
  m->levels = levels;
  m->nleaves = 1 << levels;
  m->nl = nlp;
  m->nl_min = nlmin;
  m->h = h;
  m->cmax = std::max(m->nl, 80);
  bool ok = true;
  auto A = [&](void** p, size_t bytes) {
    *p = dev_alloc(m->ctx, bytes);
    ok = ok && *p;
  };
  A((void**)&m->d_perm, rows * sizeof(int));
  A((void**)&m->d_iperm, n * sizeof(int));
  if (!uniform) A((void**)&m->d_pad2tree, rows * sizeof(int));
  A((void**)&m->d_mu, (size_t)N * sizeof(double));
  A((void**)&m->d_dst, (size_t)N * N * sizeof(double));
  if (N % 2 == 0) A((void**)&m->d_dsth, (size_t)N * N * sizeof(double));
  A((void**)&m->d_lam, 3 * (size_t)rows * sizeof(double));
  A((void**)&m->d_ws, 5 * (size_t)rows * m->cmax * sizeof(double));   // transform scratch (X, X^, 3 outputs)
  A((void**)&m->d_flags, sizeof(int));
  A((void**)&m->d_ident, (size_t)rows * m->nl * sizeof(double));
  if (!ok) {
    set_error("device allocation failed in model creation");
    hm_model_destroy(hm_);
    return HM_E_NOMEM;
  }
  hm_status st = HM_OK;
  if (!uniform) {
    // tree tables on the host: leaves in order, points row-major inside a leaf
    std::vector<int> perm(rows, -1), iperm(n, -1), pad2tree(rows, -1);
    int real = 0;
    for (int L = 0; L < (int)leaves.size(); ++L) {
      const Rect& r = leaves[L];
      int i = 0;
      for (int yy = r.y0; yy < r.y0 + r.h; ++yy)
        for (int xx = r.x0; xx < r.x0 + r.w; ++xx, ++i) {
          const int g = (dim == 2) ? yy * N + xx : xx;
          const int p = L * nlp + i;
          perm[p] = g;
          iperm[g] = p;
          pad2tree[p] = real++;
        }
    }
    if (hipMemcpy(m->d_perm, perm.data(), rows * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->d_iperm, iperm.data(), n * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->d_pad2tree, pad2tree.data(), rows * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
      set_error("model creation: copy of the tree tables failed");
      st = HM_E_DEVICE;
    }
  }
  if (st == HM_OK) st = model_tables(m);
  if (st == HM_OK) st = make_identity_stack(m);
  if (st == HM_OK) st = clear_flags(m);
  if (st == HM_OK && hipStreamSynchronize(m->stream) != hipSuccess) {
    set_error("model creation: device error");
    st = HM_E_DEVICE;
  }
  if (st != HM_OK) {
    hm_model_destroy(hm_);
    return st;
  }
  *out = hm_;
  return HM_OK;
}

}  // namespace hm

extern "C" {

hm_status hm_ctx_create(int device, void* stream, hm_alloc_fn alloc, hm_free_fn release, void* uctx,
                        hm_ctx** out) {
  if (!out) {
    set_error("out is NULL");
    return HM_E_INVAL;
  }
  *out = nullptr;
  if ((alloc == nullptr) != (release == nullptr)) {
    set_error("hm_ctx_create: give both allocator callbacks or neither");
    return HM_E_INVAL;
  }
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
    set_error("hm_ctx_create: no such device");
    return HM_E_INVAL;
  }
  hm_ctx* c = new hm_ctx();
  c->c.device = device;
  c->c.stream = (hipStream_t)stream;
  c->c.alloc = alloc;
  c->c.release = release;
  c->c.uctx = uctx;
  *out = c;
  return HM_OK;
}

void hm_ctx_destroy(hm_ctx* c) { delete c; }

hm_status hm_model_create(int device, void* stream, int dim, int N, int leaf, hm_model** out) {
  return model_create(nullptr, device, stream, dim, N, 1.0 / (N + 1), leaf, out);
}

}  // extern "C"

namespace hm {

hm_status model_create_op(Ctx* cx, int dim, const double* coords, int n, int leaf, hm_op_fn op, void* uctx,
                          bool builtin, hm_model** out, int nv) {
  if (!cx || !coords || !op || !out) {
    set_error("NULL argument");
    return HM_E_INVAL;
  }
  *out = nullptr;
  if ((dim != 1 && dim != 2) || n < 2 || leaf < 1 || nv < 1 || nv > 2 || (long)nv * n > (1 << 26)) {
    set_error("need dim in {1,2}, 2 <= n <= 2^26, leaf >= 1");
    return HM_E_INVAL;
  }
  for (long i = 0; i < (long)n * dim; ++i)
    if (!std::isfinite(coords[i])) {
      set_error("hm_model_create_op: non-finite coordinate");
      return HM_E_NONFINITE;
    }
  // the tree bisects the points; each point contributes nv rows (its variables)
  const int levels = (int)std::floor(std::log2((double)nv * n / leaf) + 1e-12);
  if (levels < 1 || levels > 20) {
    set_error("need n >= 2*leaf");
    return HM_E_INVAL;
  }
  std::vector<std::vector<int>> leaves = point_leaves(dim, coords, n, levels);
  int nlp = 0, nlmin = nv * n;
  for (const auto& v : leaves) {
    nlp = std::max(nlp, nv * (int)v.size());
    nlmin = std::min(nlmin, nv * (int)v.size());
  }
  nlp = (nlp + 3) / 4 * 4;   // rows of a leaf in groups of four (see model_create)
  const long rows = (long)nlp << levels;
  if (rows > (1L << 27)) {
    set_error("too many points");
    return HM_E_INVAL;
  }
  if (hipSetDevice(cx->device) != hipSuccess) {
    set_error("hipSetDevice failed");
    return HM_E_DEVICE;
  }
  hm_model* hm_ = new hm_model();
  Model* m = &hm_->m;
  m->ctx = cx;
  m->device = cx->device;
  m->stream = cx->stream;
  m->op_builtin = builtin;
  m->dim = dim;
  m->N = 0;
  m->n = (int)rows;
  m->n_real = nv * n;
  m->nvars = nv;
  m->nsplit = n;
  m->uniform = false;
  m->levels = levels;
  m->nleaves = 1 << levels;
  m->nl = nlp;
  m->nl_min = nlmin;
  m->h = 0.0;
  m->cmax = std::max(m->nl, 80);
  m->op = op;
  m->op_ctx = uctx;
  bool ok = true;
  auto A = [&](void** p, size_t bytes) {
    *p = dev_alloc(m->ctx, bytes);
    ok = ok && *p;
  };
  A((void**)&m->d_perm, rows * sizeof(int));
  A((void**)&m->d_iperm, (size_t)nv * n * sizeof(int));
  A((void**)&m->d_pad2tree, rows * sizeof(int));
  A((void**)&m->d_ws, 5 * (size_t)rows * m->cmax * sizeof(double));
  A((void**)&m->d_flags, sizeof(int));
  A((void**)&m->d_ident, (size_t)rows * m->nl * sizeof(double));
  A((void**)&m->d_opws, OPWS_DOUBLES * sizeof(double));
  if (!ok) {
    set_error("device allocation failed in model creation");
    hm_model_destroy(hm_);
    return HM_E_NOMEM;
  }
  // a point's nv rows are adjacent (variable 1 first); natural index v n + point
  std::vector<int> perm(rows, -1), iperm((size_t)nv * n, -1), pad2tree(rows, -1);
  int real = 0;
  for (int L = 0; L < (int)leaves.size(); ++L)
    for (int i = 0; i < (int)leaves[L].size(); ++i)
      for (int v = 0; v < nv; ++v) {
        const int g = v * n + leaves[L][i], p = L * nlp + nv * i + v;
        perm[p] = g;
        iperm[g] = p;
        pad2tree[p] = real++;
      }
  hm_status st = HM_OK;
  if (hipMemcpy(m->d_perm, perm.data(), rows * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(m->d_iperm, iperm.data(), (size_t)nv * n * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(m->d_pad2tree, pad2tree.data(), rows * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
    set_error("model creation: copy of the tree tables failed");
    st = HM_E_DEVICE;
  }
  if (st == HM_OK) st = make_identity_stack(m);
  if (st == HM_OK) st = clear_flags(m);
  if (st == HM_OK && hipStreamSynchronize(m->stream) != hipSuccess) {
    set_error("model creation: device error");
    st = HM_E_DEVICE;
  }
  if (st != HM_OK) {
    hm_model_destroy(hm_);
    return st;
  }
  *out = hm_;
  return HM_OK;
}

}  // namespace hm

extern "C" {

hm_status hm_model_create_op(hm_ctx* ctx, int dim, const double* coords, int n, int leaf, hm_op_fn op, void* uctx,
                             hm_model** out) {
  if (!ctx) {
    set_error("NULL argument");
    return HM_E_INVAL;
  }
  return model_create_op(&ctx->c, dim, coords, n, leaf, op, uctx, false, out);
}

hm_status hm_model_create_spde(hm_ctx* ctx, int dim, int nx, int ny, double h, int nvars, const int* obs_idx,
                               long long nobs, int leaf, hm_model** out) {
  if (!ctx || !out) {
    set_error("NULL argument");
    return HM_E_INVAL;
  }
  *out = nullptr;
  if (dim == 1 && ny != 1) {
    set_error("hm_model_create_spde: a one-dimensional grid has ny = 1");
    return HM_E_INVAL;
  }
  if (dim == 2 && nx != ny) {
    set_error("hm_model_create_spde: grids with nx != ny are not supported");
    return HM_E_INVAL;
  }
  if (nvars != 1 && nvars != 2) {
    set_error("hm_model_create_spde: nvars must be 1 or 2");
    return HM_E_INVAL;
  }
  if (nvars == 2) {
    if (obs_idx != nullptr || nobs != 0) {
      set_error("hm_model_create_spde: observation selections of the bivariate model are not supported");
      return HM_E_INVAL;
    }
    return model_create_bivariate(&ctx->c, dim, nx, h, leaf, out);
  }
  if (obs_idx != nullptr || nobs != 0) {
    if (!obs_idx || nobs <= 0) {
      set_error("hm_model_create_spde: obs_idx and nobs must be given together");
      return HM_E_INVAL;
    }
    if (!(h > 0.0) || !std::isfinite(h)) {
      set_error("hm_model_create_spde: need h > 0");
      return HM_E_INVAL;
    }
    return model_create_selection(&ctx->c, dim, nx, h, obs_idx, (long)nobs, leaf, out);
  }
  return model_create(&ctx->c, ctx->c.device, ctx->c.stream, dim, nx, h, leaf, out);
}

void hm_model_destroy(hm_model* mm) {
  if (!mm) return;
  Model* m = &mm->m;
  (void)hipStreamSynchronize(m->stream);
  if (m->op_release) m->op_release(m);
  for (hipEvent_t e : m->ev_pool) (void)hipEventDestroy(e);
  void* ps[] = {m->d_perm, m->d_iperm, m->d_pad2tree, m->d_dst, m->d_dsth, m->d_mu, m->d_lam, m->d_ws, m->d_flags,
                m->d_ident, m->d_red, m->d_opws};
  for (void* p : ps) dev_free(m->ctx, p);
  delete mm;
}

hm_status hm_model_info(const hm_model* mm, int* n, int* levels, int* leaf) {
  if (!mm) {
    set_error("model is NULL");
    return HM_E_INVAL;
  }
  if (n) *n = mm->m.n_real;
  if (levels) *levels = mm->m.levels;
  if (leaf) *leaf = mm->m.nl;
  return HM_OK;
}

hm_status hm_model_rows(const hm_model* mm, int* rows) {
  if (!mm || !rows) {
    set_error("NULL argument");
    return HM_E_INVAL;
  }
  *rows = mm->m.n;
  return HM_OK;
}

hm_status hm_model_set_stream(hm_model* mm, void* stream) {
  if (!mm) {
    set_error("model is NULL");
    return HM_E_INVAL;
  }
  Model* m = &mm->m;
  HM_HIP(hipStreamSynchronize(m->stream));
  m->stream = (hipStream_t)stream;
  return HM_OK;
}

hm_status hm_model_autotune(hm_model* mm, int kc, double* report) {
  if (!mm) {
    set_error("model is NULL");
    return HM_E_INVAL;
  }
  return autotune(&mm->m, kc, report);
}

hm_status hm_model_tuning(hm_model* mm, int* expand_variant, long long* reduce_split_below, int set) {
  if (!mm || !expand_variant || !reduce_split_below) {
    set_error("NULL argument");
    return HM_E_INVAL;
  }
  Model* m = &mm->m;
  if (set) {
    if (*expand_variant < 0 || *expand_variant > 3 || *reduce_split_below < 0) {
      set_error("hm_model_tuning: expand_variant in 0..3, reduce_split_below >= 0");
      return HM_E_INVAL;
    }
    m->tune_expand_rb = *expand_variant;
    m->tune_reduce_nw4 = (long)*reduce_split_below;
  } else {
    *expand_variant = m->tune_expand_rb;
    *reduce_split_below = m->tune_reduce_nw4;
  }
  return HM_OK;
}

hm_status hm_model_perm(const hm_model* mm, int* perm_host) {
  if (!mm || !perm_host) {
    set_error("NULL argument");
    return HM_E_INVAL;
  }
  const Model* m = &mm->m;
  HM_HIP(hipStreamSynchronize(m->stream));
  HM_HIP(hipMemcpy(perm_host, m->d_perm, m->n * sizeof(int), hipMemcpyDeviceToHost));   // rows entries
  return HM_OK;
}

hm_status hm_kapply(hm_model* mm, const double* theta_full, const double* X, int ldx, int c, double* Y, int ldy,
                    int which) {
  if (!mm || !X || !Y) {
    set_error("NULL argument");
    return HM_E_INVAL;
  }
  Model* m = &mm->m;
  HM_CHECK(check_theta(m, theta_full));
  if (c < 0 || ldx < m->n || ldy < m->n || which < 0 || which > 2) {
    set_error("hm_kapply: bad c, leading dimension (rows of the tree layout) or operator");
    return HM_E_INVAL;
  }
  return kapply(m, theta_full, X, ldx, c, which == 0 ? Y : nullptr, which == 1 ? Y : nullptr,
                which == 2 ? Y : nullptr, ldy);
}

hm_status hm_sketch_create(hm_model* mm, const double* omega, int rank, int oversample, const double* theta0_full,
                           hm_sketch** out) {
  return hm_sketch_create_tol(mm, omega, rank, oversample, 1e-10, theta0_full, out);
}

hm_status hm_sketch_create_tol(hm_model* mm, const double* omega, int rank, int oversample, double rank_tol,
                               const double* theta0_full, hm_sketch** out) {
  if (!mm || !omega || !out) {
    set_error("NULL argument");
    return HM_E_INVAL;
  }
  *out = nullptr;
  if (!(rank_tol >= 0.0 && rank_tol < 1.0)) {
    set_error("rank_tol must lie in [0, 1)");
    return HM_E_INVAL;
  }
  HM_CHECK(check_theta(&mm->m, theta0_full));
  if (rank < 1 || rank > 64 || oversample < 0 || rank + oversample > 80) {
    set_error("need 1 <= rank <= 64 and rank + oversample <= 80");
    return HM_E_INVAL;
  }
  Model* m = &mm->m;
  if (rank + oversample > m->nl_min) {
    set_error("rank + oversample exceeds the smallest leaf size");
    return HM_E_INVAL;
  }
  hm_sketch* hs = new hm_sketch();
  Sketch* s = &hs->s;
  s->m = m;
  s->rank = rank;
  s->rank_tol = rank_tol;
  s->oversample = oversample;
  s->ell = rank + oversample;
  const int nint = (1 << m->levels) - 1;
  s->d_k = (int*)dev_alloc(m->ctx, nint * sizeof(int));
  if (!s->d_k) {
    delete hs;
    set_error("device allocation failed");
    return HM_E_NOMEM;
  }
  hm_status st = clear_flags(m);
  if (st == HM_OK) st = sketch_build(s, omega, theta0_full);
  if (st != HM_OK) {
    hm_sketch_destroy(hs);
    return st;
  }
  *out = hs;
  return HM_OK;
}

void hm_sketch_destroy(hm_sketch* hs) {
  if (!hs) return;
  (void)hipStreamSynchronize(hs->s.m->stream);
  dev_free(hs->s.m->ctx, hs->s.d_XR);
  dev_free(hs->s.m->ctx, hs->s.d_k);
  delete hs;
}

hm_status hm_sketch_ranks(const hm_sketch* hs, int* k_host, int* kc) {
  if (!hs) {
    set_error("sketch is NULL");
    return HM_E_INVAL;
  }
  if (k_host) std::copy(hs->s.kblk.begin(), hs->s.kblk.end(), k_host);
  if (kc) *kc = hs->s.kc;
  return HM_OK;
}

void hm_H_destroy(hm_H* hh) {
  if (!hh) return;
  if (hh->h.m) (void)hipStreamSynchronize(hh->h.m->stream);
  for (void* p : hh->h.allocs) dev_free(hh->h.m->ctx, p);
  if (hh->h.h_scal) (void)hipHostFree(hh->h.h_scal);
  if (hh->h.h_flags) (void)hipHostFree(hh->h.h_flags);
  for (auto& p : hh->h.ph) {
    for (auto& pr : p.pending) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
    if (p.open) (void)hipEventDestroy(p.open);
  }
  for (hipEvent_t e : hh->h.ev_free) (void)hipEventDestroy(e);
  delete hh;
}

hm_status hm_H_create(hm_sketch* hs, int p, const int* free_idx, hm_H** out) {
  if (!hs || !out || (p > 0 && !free_idx) || p < 0 || p > nparams(hs->s.m)) {
    set_error("bad arguments to hm_H_create");
    return HM_E_INVAL;
  }
  *out = nullptr;
  hm_H* hh = new hm_H();
  HState* h = &hh->h;
  h->s = &hs->s;
  h->m = hs->s.m;
  Model* m = h->m;
  h->p = p;
  h->kc = hs->s.kc;
  bool seen[5] = {false, false, false, false, false};
  const int np = nparams(m);
  for (int q = 0; q < p; ++q) {
    int k = free_idx[q];
    if (k < 0 || k >= np || seen[k]) {
      delete hh;
      set_error(np == 5 ? "free_idx entries must be distinct values in 0..4" :
                          "free_idx entries must be distinct values in 0..3");
      return HM_E_INVAL;
    }
    seen[k] = true;
    h->pidx[q] = k;
    h->pb[q].kind = k;
    if (k <= 1) {
      h->realpos[q] = h->nreal;
      h->realidx[h->nreal++] = k;
    }
  }
  const int n = m->n, kc = h->kc, levels = m->levels, nl = m->nl;
  const size_t pset = (size_t)n * levels * kc;
  const size_t lset = (size_t)m->nleaves * nl * nl;
  const size_t nodes = (size_t)(2 << levels) - 1;
  const size_t nint = (size_t)(1 << levels) - 1;
  const size_t s2 = (size_t)kc * kc, m2 = 4 * s2;
  const size_t nk = (size_t)n * kc;
  hm_status st = HM_OK;
#define AL(ptr, cnt) \
  if (st == HM_OK) st = dalloc(h, &(ptr), (cnt))
  h->ps.bw = kc;
  AL(h->ps.F, pset);
  AL(h->D, lset);
  for (int j = 0; j < h->nreal; ++j) {
    AL(h->ps.dF[j], pset);
    AL(h->dDr[j], lset);
  }
  // factorisation
  FactorCtx& f = h->f;
  f.m = m;
  f.kc = kc;
  f.F = h->ps.F;
  f.D = h->D;
  AL(f.G, pset);
  AL(f.Dinv, lset);
  AL(f.work_leaf, lset);
  AL(f.Nn, nint * m2);
  AL(f.Sn, nodes * s2);
  AL(f.logdet_leaf, (size_t)m->nleaves);
  AL(f.logdet_node, nint);
  const size_t wT = (size_t)kc * std::max(1, levels - 1) * kc;
  AL(f.nT, nodes * wT);
  AL(f.nU, nodes * 2 * wT);
  AL(f.Ncc, nodes * s2);
  AL(f.Nx, nodes * s2);
  AL(f.tmp_panel, pset);
  // per-parameter buffers (the scale parameters alias what they share with K~)
  bool any_scale = false;
  for (int q = 0; q < p; ++q) any_scale |= (h->pb[q].kind >= 2);
  if (any_scale) AL(h->GtG, nodes * s2);
  for (int q = 0; q < p; ++q) {
    ParamBufs& pb = h->pb[q];
    if (pb.kind <= 1) {
      pb.dF = h->ps.dF[h->realpos[q]];
      pb.dD = h->dDr[h->realpos[q]];
    } else {
      AL(pb.dF, pset);
      AL(pb.dD, lset);
    }
    if (pb.kind == 2 && m->nvars == 1) {   // Xi = G, Y = Dinv (restricted to the real rows), Psi = G^T G
      pb.Xi = f.G;
      if (m->uniform) pb.Y = f.Dinv;
      else AL(pb.Y, lset);
      pb.Psi = h->GtG;
    } else {
      AL(pb.Xi, pset);
      AL(pb.Y, lset);
      AL(pb.Psi, nodes * s2);
    }
    AL(pb.dG, pset);
    AL(pb.Gh, pset);
    AL(pb.Hh, pset);
    AL(pb.E, nodes * s2);
    AL(pb.W, nodes * s2);
    AL(pb.Vt, nodes * s2);
    AL(pb.PsiP, nint * m2);
    AL(pb.Lam, nint * m2);
  }
  AL(h->node_t, nint * m2);
  AL(h->node_s, nodes * s2);
  // construction workspace
  LevelBufs& b = h->lb;
  AL(b.Y, (1 + h->nreal) * nk);   // Y | dY[0] | dY[1] adjacent (one mask launch)
  // XS | XdS[0] | XdS[1] and Z | Zq[0] | Zq[1] adjacent, so the second pass applies K to
  // all of them in one K-apply
  AL(b.XS, (1 + h->nreal) * nk);
  AL(b.Z, (1 + h->nreal) * nk);
  AL(b.Qt, nk);
  for (int j = 0; j < h->nreal; ++j) {
    if (b.Y) b.dY[j] = b.Y + (j + 1) * nk;
    if (b.XS) b.XdS[j] = b.XS + (j + 1) * nk;
    AL(b.dZ[j], nk);
    if (b.Z) b.Zq[j] = b.Z + (j + 1) * nk;
  }
  AL(b.Zl, (size_t)n * nl);
  for (int j = 0; j < h->nreal; ++j) AL(b.dZl[j], (size_t)n * nl);
  NodeBufs& nb = h->nb;
  const size_t tw = (size_t)kc * std::max(kc, nl);
  AL(nb.t, nodes * tw);
  for (int j = 0; j < h->nreal; ++j) AL(nb.dt[j], nodes * tw);
  double** smalls[] = {&nb.g, &nb.r1, &nb.r1i, &nb.r2, &nb.r2i, &nb.r3, &nb.r3i, &nb.rinv, &nb.w, &nb.mfold};
  for (double** q : smalls) AL(*q, nodes * s2);
  // reverse sweep
  AL(h->adj.Fb, pset);
  AL(h->adj.Gs, pset);
  AL(h->adj.Zb, (size_t)n * nl);
  AL(h->adj.wmode, (size_t)wmode_doubles(m));   // per-mode weights (an operator's may use two sets and a sum)
  AL(h->adj.tmpK, nk);
  AL(h->adj.uT, nodes * tw);
  AL(h->ytree, (size_t)n);
  AL(h->z, (size_t)n);
  AL(h->r, (size_t)n);
  AL(h->v, (size_t)n);
  AL(h->d_scal, (size_t)NSCAL);
  AL(h->d_part, (size_t)1024 * 16);
  h->solve_w = std::min(16, solve_max_cols(h->f));
  for (int q = 0; q < 4; ++q) AL(h->sb[q], (size_t)n * h->solve_w);
#undef AL
  if (st == HM_OK && (hipHostMalloc((void**)&h->h_scal, NSCAL * sizeof(double), hipHostMallocDefault) != hipSuccess ||
                      hipHostMalloc((void**)&h->h_flags, sizeof(int), hipHostMallocDefault) != hipSuccess)) {
    set_error("pinned host allocation failed");
    st = HM_E_NOMEM;
  }
  if (st == HM_OK) {
    // partial buffer of tree_reduce: the largest (leaves x depths x wa x wx) used per iteration
    size_t need = (size_t)m->nleaves * levels * kc * std::max(kc, nl);
    need = std::max(need, (size_t)m->nleaves * std::max(1, levels - 1) * kc * std::max(1, levels - 1) * kc);
    need = std::max(need, (size_t)m->nleaves * levels * kc * kc);
    st = ensure_reduce_ws(m, need);
  }
  if (st != HM_OK) {
    hm_H_destroy(hh);
    return st;
  }
  *out = hh;
  return HM_OK;
}

hm_status hm_build(hm_H* hh, const double* theta_full) {
  if (!hh) {
    set_error("H is NULL");
    return HM_E_INVAL;
  }
  return build_enqueue(&hh->h, theta_full, true);
}

hm_status hm_factor(hm_H* hh) {
  if (!hh) {
    set_error("H is NULL");
    return HM_E_INVAL;
  }
  HState* h = &hh->h;
  if (h->state < 1) {
    set_error("hm_factor before hm_build");
    return HM_E_STATE;
  }
  HM_CHECK(factor_enqueue(h));
  HM_CHECK(fetch_scalars(h, 0, SC_ITER_END));
  HM_CHECK(sync_check(h, true));
  phase_drain(h, false);
  return HM_OK;
}

hm_status hm_logdet(hm_H* hh, double* out) {
  if (!hh || !out) {
    set_error("NULL argument");
    return HM_E_INVAL;
  }
  HState* h = &hh->h;
  if (h->state < 2) {
    set_error("hm_logdet before hm_factor");
    return HM_E_STATE;
  }
  HM_CHECK(fetch_scalars(h, 100, 2));
  HM_HIP(hipStreamSynchronize(h->m->stream));
  *out = h->h_scal[SC_LD] + h->h_scal[SC_LD + 1];
  return HM_OK;
}

hm_status hm_solve(hm_H* hh, const double* y, double* x, long long nrhs, long long ld) {
  if (!hh || (nrhs > 0 && (!y || !x))) {
    set_error("NULL argument");
    return HM_E_INVAL;
  }
  HState* h = &hh->h;
  Model* m = h->m;
  if (nrhs < 0 || (nrhs > 0 && ld < m->n_real)) {
    set_error("hm_solve: need nrhs >= 0 and ld >= n");
    return HM_E_INVAL;
  }
  if (h->state < 2) {
    set_error("hm_solve before hm_factor");
    return HM_E_STATE;
  }
  m->mixed = h->precision;
  const int n = m->n;
  phase_begin(h, PH_SOLVE);
  for (long long c0 = 0; c0 < nrhs; c0 += h->solve_w) {
    const int w = (int)std::min<long long>(h->solve_w, nrhs - c0);
    const long cnt = (long)n * w;
    hipLaunchKernelGGL(k_permute_cols, dim3(ceil_div(cnt, 256)), dim3(256), 0, m->stream, y + c0 * ld, (long)ld,
                       h->sb[0], (long)n, m->d_perm, n, w, 1);
    HM_LAUNCH_CHECK();
    HM_CHECK(solve_refined_w(h, h->sb[0], h->sb[1], h->sb[2], h->sb[3], w));
    hipLaunchKernelGGL(k_permute_cols, dim3(ceil_div(cnt, 256)), dim3(256), 0, m->stream, h->sb[1], (long)n,
                       x + c0 * ld, (long)ld, m->d_perm, n, w, 0);
    HM_LAUNCH_CHECK();
  }
  phase_end(h, PH_SOLVE);
  h->solve_rhs += nrhs;
  return HM_OK;
}

hm_status hm_loglik_grad(hm_H* hh, const double* y, double* loglik, double* grad) {
  if (!hh || !y || !loglik) {
    set_error("NULL argument");
    return HM_E_INVAL;
  }
  HState* h = &hh->h;
  if (h->state < 2) {
    set_error("hm_loglik_grad before hm_factor");
    return HM_E_STATE;
  }
  if (grad && h->p > 0) HM_CHECK(need_deriv(h, "hm_loglik_grad"));
  HM_CHECK(loglik_enqueue(h, y, grad != nullptr));
  HM_CHECK(fetch_scalars(h, 0, SC_ITER_END));
  HM_HIP(hipStreamSynchronize(h->m->stream));
  phase_drain(h, false);
  return loglik_collect(h, loglik, grad);
}

hm_status hm_fisher(hm_H* hh, double* fim) {
  if (!hh || !fim) {
    set_error("NULL argument");
    return HM_E_INVAL;
  }
  HState* h = &hh->h;
  if (h->state < 2) {
    set_error("hm_fisher before hm_factor");
    return HM_E_STATE;
  }
  if (h->p == 0) return HM_OK;
  HM_CHECK(need_deriv(h, "hm_fisher"));
  HM_CHECK(fisher_enqueue(h));
  HM_CHECK(fetch_scalars(h, 0, SC_ITER_END));
  HM_HIP(hipStreamSynchronize(h->m->stream));
  phase_drain(h, false);
  return fisher_collect(h, fim);
}

hm_status hm_iteration(hm_H* hh, const double* theta_full, const double* y, double* loglik, double* grad,
                       double* fim) {
  if (!hh || !y || !loglik) {
    set_error("NULL argument");
    return HM_E_INVAL;
  }
  HState* h = &hh->h;
  HM_CHECK(iteration_enqueue(h, theta_full, y, grad != nullptr, fim != nullptr));
  return iteration_collect(h, loglik, grad, fim);
}

hm_status hm_iteration_batched(int nf, hm_H* const* hs, const double* thetas, const double* const* ys,
                               double* loglik, double* grad, double* fim) {
  if (nf < 0 || (nf > 0 && (!hs || !thetas || !ys || !loglik))) {
    set_error("bad arguments to hm_iteration_batched");
    return HM_E_INVAL;
  }
  for (int f = 0; f < nf; ++f) {
    if (!hs[f] || !ys[f]) {
      set_error("hm_iteration_batched: field " + std::to_string(f) + " has a NULL handle or sample");
      return HM_E_INVAL;
    }
    if (hs[f]->h.m->nvars != 1) {
      set_error("hm_iteration_batched: fields take four-entry theta (one variable per location)");
      return HM_E_INVAL;
    }
    for (int g = 0; g < f; ++g)
      if (hs[g] == hs[f]) {
        set_error("hm_iteration_batched: a handle appears twice");
        return HM_E_INVAL;
      }
  }
  // enqueue every field on its own model's stream, then collect; no host
  // synchronisation until the collect phase, so the streams run concurrently
  for (int f = 0; f < nf; ++f) {
    hm_status st = iteration_enqueue(&hs[f]->h, thetas + 4L * f, ys[f], grad != nullptr, fim != nullptr);
    if (st != HM_OK) {
      set_error("field " + std::to_string(f) + ": " + get_error());
      for (int g = 0; g < f; ++g) (void)hipStreamSynchronize(hs[g]->h.m->stream);
      return st;
    }
  }
  hm_status first = HM_OK;
  std::string msg;
  long go = 0, fo = 0;
  for (int f = 0; f < nf; ++f) {
    HState* h = &hs[f]->h;
    hm_status st = iteration_collect(h, loglik + f, grad ? grad + go : nullptr, fim ? fim + fo : nullptr);
    if (st != HM_OK && first == HM_OK) {
      first = st;
      msg = "field " + std::to_string(f) + ": " + get_error();
    }
    go += h->p;
    fo += (long)h->p * h->p;
  }
  if (first != HM_OK) set_error(msg);
  return first;
}

hm_status hm_H_set_precision(hm_H* hh, int precision) {
  if (!hh || precision < 0 || precision > 2) {
    set_error("precision must be 0 (FP64), 1 (mixed: FP32 panel products) or 2 (mixed with BF16 trace panels)");
    return HM_E_INVAL;
  }
  hh->h.precision = precision;
  hh->h.state = 0;   // factors of the other precision are not reused
  hh->h.have_deriv = false;
  return HM_OK;
}

hm_status hm_loglik(hm_H* hh, const double* theta_full, const double* y, double* loglik) {
  if (!hh || !y || !loglik) {
    set_error("NULL argument");
    return HM_E_INVAL;
  }
  HState* h = &hh->h;
  // K~ only: neither L~ nor the reverse sweep needs the derivative matrices
  HM_CHECK(build_enqueue(h, theta_full, false));
  HM_CHECK(factor_enqueue(h));
  HM_CHECK(loglik_enqueue(h, y, false));
  HM_CHECK(fetch_scalars(h, 0, SC_ITER_END));
  HM_CHECK(sync_check(h, true));
  phase_drain(h, false);
  return loglik_collect(h, loglik, nullptr);
}

hm_status hm_grad_reverse(hm_H* hh, double* grad) {
  if (!hh || !grad) {
    set_error("NULL argument");
    return HM_E_INVAL;
  }
  HState* h = &hh->h;
  Model* m = h->m;
  if (h->state < 2 || h->z_gen != h->gen) {
    set_error("hm_grad_reverse: needs the K~^{-1} y of the current factorisation (call hm_loglik first)");
    return HM_E_STATE;
  }
  if (h->p == 0) return HM_OK;
  m->mixed = h->precision;
  phase_begin(h, PH_REVERSE);
  h->reverse_sweeps += 1;
  HM_CHECK(node_prep(h->f));
  HM_CHECK(adjoint_init(h->f, h->z, h->adj));
  HM_CHECK(adjoint_sweep(m, h->theta, h->s, h->ps, h->lb, h->nb, h->adj));
  if (m->op_vjp_final) {
    HM_CHECK(m->op_vjp_final(m, h->theta, h->adj.wmode, h->d_scal + SC_ADJ));
  } else if (m->op) {
    // the operator's vector-Jacobian products were summed directly (see kvjp; the fifth
    // sum, the second variable's part of <Ybar, X>, for the bivariate model)
    HM_HIP(hipMemcpyAsync(h->d_scal + SC_ADJ, h->adj.wmode, 5 * sizeof(double), hipMemcpyDeviceToDevice,
                          m->stream));
  } else {
    const long NN = (long)m->N * (m->dim == 2 ? m->N : 1);   // modes of the transforms
    const double* wv[1] = {h->adj.wmode};
    const double* lv[3] = {m->d_lam, m->d_lam + NN, m->d_lam + 2 * NN};
    HM_CHECK(dots(m, wv, 1, lv, 3, NN, h->d_scal + SC_ADJ, h->d_part));
    HM_CHECK(sum_scalar(m, h->adj.wmode, NN, 0, h->d_scal + SC_ADJ + 3, h->d_part));
  }
  phase_end(h, PH_REVERSE);
  HM_CHECK(fetch_scalars(h, SC_ADJ, 5));
  HM_CHECK(sync_check(h, true));
  phase_drain(h, false);
  // w-weighted mode sums: <w, lambda>, <w, dlambda/dkappa>, <w, dlambda/dalpha>, sum w
  // (lambda: the physics part of the mode multiplier, sigma2 times the unit-scale one,
  // so de/dsigma2 = lambda / sigma2; de/dtau2 = 1).  Bivariate model: sum w splits into
  // the two variables' nuggets, t[4] the second variable's part.
  const double* t = h->h_scal + SC_ADJ;
  const double sigma2 = h->theta[3];
  const bool two = m->nvars == 2;
  const double tb[5] = {t[1], t[2], two ? t[3] - t[4] : t[3], t[0] / sigma2, two ? t[4] : 0.0};
  for (int q = 0; q < h->p; ++q) {
    grad[q] = tb[h->pidx[q]];
    if (!std::isfinite(grad[q])) {
      set_error("non-finite gradient");
      return HM_E_NONFINITE;
    }
  }
  return HM_OK;
}

hm_status hm_loglik_grad_adjoint(hm_H* hh, const double* theta_full, const double* y, double* loglik,
                                 double* grad) {
  HM_CHECK(hm_loglik(hh, theta_full, y, loglik));
  if (grad) HM_CHECK(hm_grad_reverse(hh, grad));
  return HM_OK;
}

hm_status hm_stats(hm_H* hh, void* out, size_t bytes) {
  if (!hh || !out) {
    set_error("NULL argument");
    return HM_E_INVAL;
  }
  HState* h = &hh->h;
  HM_HIP(hipStreamSynchronize(h->m->stream));
  phase_drain(h, true);
  hm_stats_t st{};
  const ModelCounters& c = h->m->cnt;
  st.kapply_calls = c.kapply_calls;
  st.kapply_columns = c.kcols_value;
  st.kapply_deriv_columns = c.kcols_deriv;
  st.builds = h->builds;
  st.deriv_builds = h->deriv_builds;
  st.factors = h->factors;
  st.loglik_evals = h->loglik_evals;
  st.grad_evals = h->grad_evals;
  st.reverse_sweeps = h->reverse_sweeps;
  st.fisher_evals = h->fisher_evals;
  st.solve_rhs = h->solve_rhs;
  st.ms_build = h->ph[PH_BUILD].ms;
  st.ms_factor = h->ph[PH_FACTOR].ms;
  st.ms_loglik = h->ph[PH_LOGLIK].ms;
  st.ms_fisher = h->ph[PH_FISHER].ms;
  st.ms_reverse = h->ph[PH_REVERSE].ms;
  st.ms_solve = h->ph[PH_SOLVE].ms;
  st.device_bytes = (long long)h->dev_bytes;
  std::memcpy(out, &st, std::min(bytes, sizeof(st)));
  return HM_OK;
}

hm_status hm_stats_reset(hm_H* hh) {
  if (!hh) {
    set_error("H is NULL");
    return HM_E_INVAL;
  }
  HState* h = &hh->h;
  HM_HIP(hipStreamSynchronize(h->m->stream));
  phase_drain(h, true);
  for (auto& p : h->ph) p.ms = 0.0;
  h->builds = h->deriv_builds = h->factors = h->loglik_evals = h->grad_evals = h->fisher_evals = 0;
  h->reverse_sweeps = h->solve_rhs = 0;
  h->m->cnt = ModelCounters{};
  return HM_OK;
}

hm_status hm_export(hm_H* hh, int what, double* dst) {
  if (!hh || !dst) {
    set_error("NULL argument");
    return HM_E_INVAL;
  }
  HState* h = &hh->h;
  if (h->state < 1) {
    set_error("hm_export before hm_build");
    return HM_E_STATE;
  }
  Model* m = h->m;
  const size_t pset = (size_t)m->n * m->levels * h->kc;
  const size_t lset = (size_t)m->nleaves * m->nl * m->nl;
  const double* src = nullptr;
  size_t cnt = 0;
  if (what == 0) { src = h->ps.F; cnt = pset; }
  else if (what >= 1 && what <= 2 && what - 1 < h->nreal) { src = h->ps.dF[what - 1]; cnt = pset; }
  else if (what == 10) { src = h->D; cnt = lset; }
  else if (what >= 11 && what <= 12 && what - 11 < h->nreal) { src = h->dDr[what - 11]; cnt = lset; }
  else {
    set_error("hm_export: unknown item");
    return HM_E_INVAL;
  }
  HM_HIP(hipMemcpyAsync(dst, src, cnt * sizeof(double), hipMemcpyDeviceToDevice, m->stream));
  HM_HIP(hipStreamSynchronize(m->stream));
  return HM_OK;
}

hm_status hm_profile_enable(hm_model* mm, int family) {
  if (!mm || family < -1 || family >= PF_COUNT) {
    set_error("bad profiling family");
    return HM_E_INVAL;
  }
  Model* m = &mm->m;
  HM_HIP(hipStreamSynchronize(m->stream));
  m->prof.clear();
  m->ev_used = 0;
  m->prof_family = family;
  return HM_OK;
}

hm_status hm_profile_read(hm_model* mm, double* ms, long long* launches, double* flops, double* bytes) {
  if (!mm) {
    set_error("model is NULL");
    return HM_E_INVAL;
  }
  Model* m = &mm->m;
  HM_HIP(hipStreamSynchronize(m->stream));
  double t = 0.0, fl = 0.0, by = 0.0;
  for (const ProfRec& r : m->prof) {
    float e = 0.0f;
    if (r.a && r.b && hipEventElapsedTime(&e, r.a, r.b) == hipSuccess) t += e;
    fl += r.flops;
    by += r.bytes;
  }
  if (ms) *ms = t;
  if (launches) *launches = (long long)m->prof.size();
  if (flops) *flops = fl;
  if (bytes) *bytes = by;
  return HM_OK;
}

}  // extern "C"
