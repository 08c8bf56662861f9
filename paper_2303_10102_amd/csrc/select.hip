// Observations of a subset of the grid (Sec. 5.1, eq. "projection", with the observation
// operator a selection Phi of grid nodes; Sec. 5.2.1 forms its smaller data sets by
// subsampling the grid this way):
//   K_obs = sigma2 Phi M M^T Phi^T + tau2 I,   M = A^{-1} B^{-1} on the full grid,
// the nugget on the observations only.  The model is an operator model over the
// observed points (their KD-tree, padded leaves); its operator scatters a block of
// columns onto the full grid (zero at unobserved nodes), applies the full-grid stencil
// model's sine-transform K-apply (value or one derivative, unit sigma2, no nugget) and
// reads the observed nodes back.  The reverse sweep scatters both the columns and
// their adjoints and accumulates the full-grid model's per-mode products, so the
// parameter sums use the mode multipliers of the full grid.
#include <cmath>
#include <vector>

#include "hm_internal.h"
#include "hm_trace.h"

namespace hm {

hm_status kapply_ws(Model* m, double* ws, int cblk, const double* theta, const double* X, int ldx, int c,
                    double* outK, double* outKap, double* outAlp, int ldo);
hm_status kvjp(Model* m, const double* theta, const double* X, int ldx, const double* Yb, int ldb, int c,
               double* wmode);
hm_status ensure_scale(Model* m, const double* theta);

struct SelOp {
  hm_model* grid = nullptr;    // the full-grid stencil model
  Model* outer = nullptr;
  int* d_obs_at = nullptr;     // grid tree row -> observation index (-1: unobserved or padding)
  int* d_row_of = nullptr;     // observation index -> grid tree row
  int* d_tree_at = nullptr;    // grid tree row -> tree row of the observation model (-1 elsewhere)
  double* Xg = nullptr;        // grid rows x cmax (outer): columns on the full grid
  double* Yg = nullptr;
  long nobs = 0;
  int cmax = 0;
};

// G[r + j ldg] = src[r] >= 0 ? X[src[r] + j ldx] : 0   (a block onto the full grid)
__global__ void __launch_bounds__(256) k_sel_spread(double* G, long ldg, const double* X, long ldx, const int* src,
                                                    long rows, int c) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * c) return;
  const long r = e % rows, j = e / rows;
  const int s = src[r];
  G[r + j * ldg] = s >= 0 ? X[s + j * ldx] : 0.0;
}
// Y[i + j ldy] = G[row[i] + j ldg]   (the observed nodes read back)
__global__ void __launch_bounds__(256) k_sel_read(double* Y, long ldy, const double* G, long ldg, const int* row,
                                                  long nobs, int c) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nobs * c) return;
  const long i = e % nobs, j = e / nobs;
  Y[i + j * ldy] = G[row[i] + j * ldg];
}

static int sel_apply(void* uctx, int which, const double* theta, const double* X, long long ldx, long long cc,
                     double* Y, long long ldy, void* stream) {
  SelOp* s = (SelOp*)uctx;
  Model* g = &s->grid->m;
  const int c = (int)cc;
  if (!(theta[0] > 0.0) || !(theta[1] >= 0.0)) {
    set_error("theta must satisfy kappa > 0, alpha >= 0, tau2 > 0, sigma2 > 0");
    return HM_E_INVAL;
  }
  if (c > s->cmax || ldx < s->nobs || ldy < s->nobs || which < 0 || which > 2) {
    set_error("observation-subset operator: unexpected block shape");
    return HM_E_INVAL;
  }
  g->stream = (hipStream_t)stream;
  const long rows = g->n;
  hipLaunchKernelGGL(k_sel_spread, dim3(ceil_div(rows * c, 256)), dim3(256), 0, g->stream, s->Xg, rows, X, (long)ldx,
                     s->d_obs_at, rows, c);
  HM_LAUNCH_CHECK();
  const double unit[4] = {theta[0], theta[1], 0.0, 1.0};   // K_op: unit sigma2, no nugget
  double* outs[3] = {nullptr, nullptr, nullptr};
  outs[which] = s->Yg;
  HM_CHECK(kapply_ws(g, g->d_ws, g->cmax, unit, s->Xg, (int)rows, c, outs[0], outs[1], outs[2], (int)rows));
  hipLaunchKernelGGL(k_sel_read, dim3(ceil_div(s->nobs * c, 256)), dim3(256), 0, g->stream, Y, (long)ldy, s->Yg, rows,
                     s->d_row_of, s->nobs, c);
  HM_LAUNCH_CHECK();
  return HM_OK;
}

// per-mode products of the full-grid model for columns X and adjoints Yb in the
// observation model's tree order
static hm_status sel_vjp(Model* m, const double* theta, const double* X, int ldx, const double* Yb, int ldb, int c,
                         double* wmode) {
  SelOp* s = (SelOp*)m->op_ctx;
  Model* g = &s->grid->m;
  g->stream = m->stream;
  const long rows = g->n;
  for (int c0 = 0; c0 < c; c0 += s->cmax) {
    const int cc = std::min(s->cmax, c - c0);
    hipLaunchKernelGGL(k_sel_spread, dim3(ceil_div(rows * cc, 256)), dim3(256), 0, m->stream, s->Xg, rows,
                       X + (long)c0 * ldx, (long)ldx, s->d_tree_at, rows, cc);
    HM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sel_spread, dim3(ceil_div(rows * cc, 256)), dim3(256), 0, m->stream, s->Yg, rows,
                       Yb + (long)c0 * ldb, (long)ldb, s->d_tree_at, rows, cc);
    HM_LAUNCH_CHECK();
    HM_CHECK(kvjp(g, theta, s->Xg, (int)rows, s->Yg, (int)rows, cc, wmode));
  }
  return HM_OK;
}

// <w, lambda>, <w, dlambda/dkappa>, <w, dlambda/dalpha>, sum w over the grid's modes
static hm_status sel_vjp_final(Model* m, const double* theta, const double* wmode, double* out4) {
  SelOp* s = (SelOp*)m->op_ctx;
  Model* g = &s->grid->m;
  const long NN = (long)g->N * (g->dim == 2 ? g->N : 1);
  const double* wv[1] = {wmode};
  g->stream = m->stream;
  HM_CHECK(ensure_scale(g, theta));   // the multipliers at theta (the operator ran at unit sigma2)
  const double* lv[3] = {g->d_lam, g->d_lam + NN, g->d_lam + 2 * NN};
  double* d = m->d_opws + 1024 * 16;
  HM_CHECK(dots(m, wv, 1, lv, 3, NN, d, m->d_opws));
  HM_CHECK(sum_scalar(m, wmode, NN, 0, d + 3, m->d_opws));
  HM_HIP(hipMemcpyAsync(out4, d, 4 * sizeof(double), hipMemcpyDeviceToDevice, m->stream));
  return HM_OK;
}

static void sel_release(Model* m) {
  SelOp* s = (SelOp*)m->op_ctx;
  if (!s) return;
  void* bufs[] = {s->d_obs_at, s->d_row_of, s->d_tree_at, s->Xg, s->Yg};
  for (void* p : bufs) dev_free(m->ctx, p);
  if (s->grid) hm_model_destroy(s->grid);
  delete s;
  m->op_ctx = nullptr;
}

hm_status model_create_selection(Ctx* cx, int dim, int N, double h, const int* obs, long nobs, int leaf,
                                 hm_model** out) {
  const long full = (long)N * (dim == 2 ? N : 1);
  if (nobs < 2 || nobs > full) {
    set_error("observation selection: need 2 <= nobs <= grid points");
    return HM_E_INVAL;
  }
  std::vector<int> obs_of(full, -1);
  for (long i = 0; i < nobs; ++i) {
    if (obs[i] < 0 || obs[i] >= full) {
      set_error("observation selection: index outside the grid");
      return HM_E_INVAL;
    }
    if (obs_of[obs[i]] >= 0) {
      set_error("observation selection: repeated grid index");
      return HM_E_INVAL;
    }
    obs_of[obs[i]] = (int)i;
  }
  // the full-grid model first (its checks of dim, N, h, leaf apply)
  hm_model* gm = nullptr;
  HM_CHECK(model_create(cx, cx->device, cx->stream, dim, N, h, leaf, &gm));
  Model* g = &gm->m;
  std::vector<double> xy((size_t)nobs * dim);
  for (long i = 0; i < nobs; ++i) {
    if (dim == 2) {
      xy[2 * i] = obs[i] % N;
      xy[2 * i + 1] = obs[i] / N;
    } else {
      xy[i] = obs[i];
    }
  }
  SelOp* s = new SelOp();
  s->grid = gm;
  s->nobs = nobs;
  hm_model* mm = nullptr;
  hm_status st = model_create_op(cx, dim, xy.data(), (int)nobs, leaf, sel_apply, s, true, &mm);
  if (st != HM_OK) {
    hm_model_destroy(gm);
    delete s;
    return st;
  }
  Model* m = &mm->m;
  s->outer = m;
  s->cmax = m->cmax;
  m->op_release = sel_release;
  m->op_vjp = sel_vjp;
  m->op_vjp_final = sel_vjp_final;
  m->op_wmode = full + 8;
  // index tables: grid tree rows, observation indices, observation-model tree rows
  const long rows = g->n;
  std::vector<int> gperm(rows), operm(m->n), oiperm(nobs, -1);
  if (hipMemcpy(gperm.data(), g->d_perm, rows * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(operm.data(), m->d_perm, (size_t)m->n * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) {
    hm_model_destroy(mm);
    set_error("observation selection: copy of the tree tables failed");
    return HM_E_DEVICE;
  }
  for (int t = 0; t < m->n; ++t)
    if (operm[t] >= 0) oiperm[operm[t]] = t;
  std::vector<int> obs_at(rows, -1), row_of(nobs, -1), tree_at(rows, -1);
  for (long r = 0; r < rows; ++r) {
    const int gi = gperm[r];
    if (gi < 0) continue;
    const int i = obs_of[gi];
    if (i < 0) continue;
    obs_at[r] = i;
    row_of[i] = (int)r;
    tree_at[r] = oiperm[i];
  }
  for (long i = 0; i < nobs; ++i)
    if (row_of[i] < 0 || oiperm[i] < 0) {
      hm_model_destroy(mm);
      set_error("observation selection: a node is missing from a tree table");
      return HM_E_INVAL;
    }
  bool ok = true;
  auto A = [&](void** p, size_t bytes) {
    *p = dev_alloc(m->ctx, bytes);
    ok = ok && *p;
  };
  A((void**)&s->d_obs_at, rows * sizeof(int));
  A((void**)&s->d_row_of, (size_t)nobs * sizeof(int));
  A((void**)&s->d_tree_at, rows * sizeof(int));
  A((void**)&s->Xg, (size_t)rows * s->cmax * sizeof(double));
  A((void**)&s->Yg, (size_t)rows * s->cmax * sizeof(double));
  if (!ok) {
    hm_model_destroy(mm);
    set_error("device allocation failed in the observation-selection model");
    return HM_E_NOMEM;
  }
  if (hipMemcpy(s->d_obs_at, obs_at.data(), rows * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(s->d_row_of, row_of.data(), (size_t)nobs * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(s->d_tree_at, tree_at.data(), rows * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
    hm_model_destroy(mm);
    set_error("observation selection: copy of the index tables failed");
    return HM_E_DEVICE;
  }
  *out = mm;
  return HM_OK;
}

}  // namespace hm
