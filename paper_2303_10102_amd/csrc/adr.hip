// Advection-diffusion-reaction covariance (Sec. 5.3, eqs. "ad1", "ad2"): the field u
// solves L u = phi, L u = -kd Lap u + v . grad u + c u, whose latent source phi has
// the Matern covariance of the SPDE representation (Sec. 5.1, eq. "latent
// covariance", mass lumped): B^{-2}, B = kappa^2 I - Lap.  With a nugget,
//   K = sigma2 L^{-1} B^{-2} L^{-T} + tau2 I,   theta_full = (kappa, c, tau2, sigma2).
// Constant coefficients, central differences on the unit square, Dirichlet boundary,
// h = 1/(N+1).  L is not symmetric for v != 0, so L^{-1} and L^{-T} differ.
//
// Direct solves by a similarity transform.  Along one axis L acts as the tridiagonal
// Toeplitz T = tridiag(sub, 2 kd / h^2, sup), sub = -kd/h^2 - v/(2h),
// sup = -kd/h^2 + v/(2h).  With rho = sqrt(sup / sub) and D = diag(rho^i),
// T = D^{-1} T_s D for the symmetric T_s = tridiag(t, 2 kd/h^2, t), t = -sqrt(sub sup),
// whose eigenvectors are the orthonormal sine transform S and eigenvalues
// lambda_p = 2 kd / h^2 + 2 t cos(p pi / (N+1)).  On the grid (x fastest),
// D = D_y (x) D_x and L = D^{-1} (S (x) S) diag(Lambda) (S (x) S) D with
// Lambda_pq = lambda^x_p + lambda^y_q + c > 0, and B^{-2} = (S (x) S) diag(Lambda_B^{-2})
// (S (x) S), Lambda_B = kappa^2 + mu_p + mu_q.  Hence
//   K_op = L^{-1} B^{-2} L^{-T}
//        = (E_y^T (x) E_x^T) Lambda^{-1} (W_y (x) W_x) Lambda_B^{-2} (W_y (x) W_x) Lambda^{-1} (E_y (x) E_x)
// with E = S D^{-1} and W = S D S per axis: separable N x N transforms (batched FP64
// GEMMs on the matrix cores) around three per-mode scalings.  The transforms carry the
// conditioning of D, rho^{N-1}; the model accepts advection with rho^{+-(N-1)} <= 1e3.
// Derivatives: d/dkappa replaces Lambda_B^{-2} by -4 kappa Lambda_B^{-3};
// d/dc = -(E^T)(Lambda^{-2} M Lambda^{-1} + Lambda^{-1} M Lambda^{-2})(E), M = W Lambda_B^{-2} W.
#include <cmath>
#include <vector>

#include "hm_internal.h"
#include "hm_trace.h"

namespace hm {

struct AdrOp {
  Model* m = nullptr;
  int N = 0;
  double* E[2] = {nullptr, nullptr};   // x, y: N x N column-major, S D^{-1}
  double* W[2] = {nullptr, nullptr};   // x, y: S D S
  double* lam[2] = {nullptr, nullptr}; // x, y: eigenvalues of T_s
  double* mu = nullptr;                // eigenvalues of the 1D -Laplacian
  double* modes = nullptr;             // 4 x N^2: 1/Lambda, 1/Lambda^2, 1/Lambda_B^2, -4 kappa / Lambda_B^3
  double* w[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};   // n x cmax work buffers
  double key[2] = {NAN, NAN};
};

__global__ void k_adr_modes(double* modes, const double* lx, const double* ly, const double* mu, int N, double kappa,
                            double c) {
  const long NN = (long)N * N;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= NN) return;
  const int p = (int)(e % N), q = (int)(e / N);
  const double L = lx[p] + ly[q] + c;
  const double B = kappa * kappa + mu[p] + mu[q];
  modes[e] = 1.0 / L;
  modes[NN + e] = 1.0 / (L * L);
  modes[2 * NN + e] = 1.0 / (B * B);
  modes[3 * NN + e] = -4.0 * kappa / (B * B * B);
}
// out[e + j n] = s[e] in[e + j n] (+ out: acc = 1 adds to out; a second scaled input in2, s2)
__global__ void k_adr_scale(double* out, const double* in, const double* s, const double* in2, const double* s2,
                            long n, int c, double alpha) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * c) return;
  const long i = e % n;
  double v = s[i] * in[e];
  if (in2) v += s2[i] * in2[e];
  out[e] = alpha * v;
}

// out_j = op(Ax) in_j op(Ay)^T for the c grid columns in_j (N x N, x along rows)
static hm_status adr_sep(const AdrOp* a, hipStream_t st, const double* Ax, bool tx, const double* Ay, bool ty,
                         const double* in, double* out, double* tmp, int c) {
  const int N = a->N;
  const long NN = (long)N * N;
  HM_CHECK(gemm(st, tx, false, N, N * c, N, 1.0, Ax, N, 0, in, N, 0, 0.0, tmp, N, 0, 1));
  HM_CHECK(gemm(st, false, !ty, N, N, N, 1.0, tmp, N, NN, Ay, N, 0, 0.0, out, N, NN, c));
  return HM_OK;
}
static hm_status adr_scale(const AdrOp* a, hipStream_t st, double* out, const double* in, const double* s,
                           const double* in2, const double* s2, int c, double alpha) {
  const long NN = (long)a->N * a->N;
  hipLaunchKernelGGL(k_adr_scale, dim3(ceil_div(NN * c, 256)), dim3(256), 0, st, out, in, s, in2, s2, NN, c, alpha);
  HM_LAUNCH_CHECK();
  return HM_OK;
}

static int adr_apply(void* uctx, int which, const double* theta, const double* X, long long ldx, long long cc,
                     double* Y, long long ldy, void* stream) {
  AdrOp* a = (AdrOp*)uctx;
  hipStream_t st = (hipStream_t)stream;
  const int N = a->N, c = (int)cc;
  const long NN = (long)N * N;
  const double kappa = theta[0], creact = theta[1];
  if (!(kappa > 0.0) || !(creact >= 0.0)) {
    set_error("advection-diffusion-reaction model: need kappa > 0 and c >= 0");
    return HM_E_INVAL;
  }
  if (ldx != NN || ldy != NN || c > a->m->cmax) {
    set_error("advection-diffusion-reaction operator: unexpected block shape");
    return HM_E_INVAL;
  }
  if (!(a->key[0] == kappa && a->key[1] == creact)) {
    hipLaunchKernelGGL(k_adr_modes, dim3(ceil_div(NN, 256)), dim3(256), 0, st, a->modes, a->lam[0], a->lam[1], a->mu,
                       N, kappa, creact);
    HM_LAUNCH_CHECK();
    a->key[0] = kappa;
    a->key[1] = creact;
  }
  const double* aL = a->modes;
  const double* aL2 = a->modes + NN;
  const double* bB = a->modes + 2 * NN;
  const double* dB = a->modes + 3 * NN;
  double** w = a->w;
  const double *Ex = a->E[0], *Ey = a->E[1], *Wx = a->W[0], *Wy = a->W[1];
  HM_CHECK(adr_sep(a, st, Ex, false, Ey, false, X, w[0], w[4], c));   // (E_y (x) E_x) X
  if (which == 0 || which == 1) {
    HM_CHECK(adr_scale(a, st, w[1], w[0], aL, nullptr, nullptr, c, 1.0));
    HM_CHECK(adr_sep(a, st, Wx, false, Wy, false, w[1], w[0], w[4], c));
    HM_CHECK(adr_scale(a, st, w[1], w[0], which == 0 ? bB : dB, nullptr, nullptr, c, 1.0));
    HM_CHECK(adr_sep(a, st, Wx, false, Wy, false, w[1], w[0], w[4], c));
    HM_CHECK(adr_scale(a, st, w[1], w[0], aL, nullptr, nullptr, c, 1.0));
  } else {
    // d/dc: -(Lambda^{-2} M Lambda^{-1} + Lambda^{-1} M Lambda^{-2}), M = W Lambda_B^{-2} W
    HM_CHECK(adr_scale(a, st, w[1], w[0], aL, nullptr, nullptr, c, 1.0));    // u1
    HM_CHECK(adr_scale(a, st, w[2], w[0], aL2, nullptr, nullptr, c, 1.0));   // u2
    HM_CHECK(adr_sep(a, st, Wx, false, Wy, false, w[1], w[0], w[4], c));
    HM_CHECK(adr_scale(a, st, w[1], w[0], bB, nullptr, nullptr, c, 1.0));
    HM_CHECK(adr_sep(a, st, Wx, false, Wy, false, w[1], w[3], w[4], c));     // M u1 -> w3
    HM_CHECK(adr_sep(a, st, Wx, false, Wy, false, w[2], w[0], w[4], c));
    HM_CHECK(adr_scale(a, st, w[2], w[0], bB, nullptr, nullptr, c, 1.0));
    HM_CHECK(adr_sep(a, st, Wx, false, Wy, false, w[2], w[0], w[4], c));     // M u2 -> w0
    HM_CHECK(adr_scale(a, st, w[1], w[3], aL2, w[0], aL, c, -1.0));
  }
  HM_CHECK(adr_sep(a, st, Ex, true, Ey, true, w[1], Y, w[4], c));       // (E_y^T (x) E_x^T)
  return HM_OK;
}

// ---------------------------------------------------------------------------
// Vector-Jacobian product with the operator's mode structure (the same form as the
// stencil model's): for Y = K X and the adjoint Ybar, with u = E X, v = E Ybar,
// a = W Lambda^{-1} (.), b = W Lambda_B^{-2} a,
//   <Ybar, K_op X>            = sum_m Lambda_B^{-2} a_X a_Ybar
//   <Ybar, dK_op/dkappa X>    = sum_m (-4 kappa Lambda_B^{-3}) a_X a_Ybar
//   <Ybar, dK_op/dc X>        = -sum_m Lambda^{-2} (v b_X + u b_Ybar)
// so each call adds a_X a_Ybar to wk and v b_X + u b_Ybar to wc (per mode, summed over
// the columns), and <Ybar, X> to one scalar; the parameter sums are formed once at the
// end.  Only transforms of X and Ybar enter, no operator derivative is applied.
// ---------------------------------------------------------------------------
__global__ void k_mode_accum(double* w, const double* A1, const double* B1, const double* A2, const double* B2,
                             long NN, int c) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= NN) return;
  double s = 0.0;
  for (int j = 0; j < c; ++j) {
    const long k = e + j * NN;
    s += A1[k] * B1[k];
    if (A2) s += A2[k] * B2[k];
  }
  w[e] += s;
}
__global__ void k_add_scalar(double* w, const double* d) {
  if (threadIdx.x == 0) w[0] += d[0];
}
__global__ void k_adr_final(double* out4, const double* d, const double* tau_sum, double sigma2) {
  if (threadIdx.x == 0) {
    out4[0] = sigma2 * d[0];
    out4[1] = sigma2 * d[1];
    out4[2] = -sigma2 * d[2];
    out4[3] = tau_sum[0];
  }
}

hm_status kvjp_gather(Model* m, const double* X, int ldx, double* Xn, int c);

static hm_status adr_vjp(Model* m, const double* theta, const double* X, int ldx, const double* Yb, int ldb, int c,
                         double* wmode) {
  AdrOp* a = (AdrOp*)m->op_ctx;
  hipStream_t st = m->stream;
  const int N = a->N, n = m->n, cblk = m->cmax;
  const long NN = (long)N * N;
  double* Xn = m->d_ws;
  double* Bn = m->d_ws + (long)n * cblk;
  double* aY = m->d_ws + 2L * n * cblk;
  double** w = a->w;
  if (!(a->key[0] == theta[0] && a->key[1] == theta[1])) {
    hipLaunchKernelGGL(k_adr_modes, dim3(ceil_div(NN, 256)), dim3(256), 0, st, a->modes, a->lam[0], a->lam[1], a->mu,
                       N, theta[0], theta[1]);
    HM_LAUNCH_CHECK();
    a->key[0] = theta[0];
    a->key[1] = theta[1];
  }
  const double* aL = a->modes;
  const double* bB = a->modes + 2 * NN;
  const double *Ex = a->E[0], *Ey = a->E[1], *Wx = a->W[0], *Wy = a->W[1];
  for (int c0 = 0; c0 < c; c0 += cblk) {
    const int cc = std::min(cblk, c - c0);
    HM_CHECK(kvjp_gather(m, X + (long)c0 * ldx, ldx, Xn, cc));
    HM_CHECK(kvjp_gather(m, Yb + (long)c0 * ldb, ldb, Bn, cc));
    // <Ybar, X> for the nugget
    const double* A1[1] = {Bn};
    const double* B1[1] = {Xn};
    HM_CHECK(dots(m, A1, 1, B1, 1, NN * cc, m->d_opws + 1024 * 16, m->d_opws));
    hipLaunchKernelGGL(k_add_scalar, dim3(1), dim3(64), 0, st, wmode + 2 * NN, m->d_opws + 1024 * 16);
    HM_LAUNCH_CHECK();
    HM_CHECK(adr_sep(a, st, Ex, false, Ey, false, Xn, w[0], w[4], cc));   // u
    HM_CHECK(adr_sep(a, st, Ex, false, Ey, false, Bn, w[1], w[4], cc));   // v
    HM_CHECK(adr_scale(a, st, w[2], w[0], aL, nullptr, nullptr, cc, 1.0));
    HM_CHECK(adr_sep(a, st, Wx, false, Wy, false, w[2], w[3], w[4], cc));  // a_X
    HM_CHECK(adr_scale(a, st, w[2], w[1], aL, nullptr, nullptr, cc, 1.0));
    HM_CHECK(adr_sep(a, st, Wx, false, Wy, false, w[2], aY, w[4], cc));    // a_Ybar
    hipLaunchKernelGGL(k_mode_accum, dim3(ceil_div(NN, 256)), dim3(256), 0, st, wmode, w[3], aY, nullptr, nullptr, NN,
                       cc);
    HM_LAUNCH_CHECK();
    HM_CHECK(adr_scale(a, st, w[2], w[3], bB, nullptr, nullptr, cc, 1.0));
    HM_CHECK(adr_sep(a, st, Wx, false, Wy, false, w[2], w[3], w[4], cc));  // b_X
    HM_CHECK(adr_scale(a, st, w[2], aY, bB, nullptr, nullptr, cc, 1.0));
    HM_CHECK(adr_sep(a, st, Wx, false, Wy, false, w[2], aY, w[4], cc));    // b_Ybar
    hipLaunchKernelGGL(k_mode_accum, dim3(ceil_div(NN, 256)), dim3(256), 0, st, wmode + NN, w[1], w[3], w[0], aY, NN,
                       cc);
    HM_LAUNCH_CHECK();
  }
  return HM_OK;
}

static hm_status adr_vjp_final(Model* m, const double* theta, const double* wmode, double* out4) {
  AdrOp* a = (AdrOp*)m->op_ctx;
  const long NN = (long)a->N * a->N;
  const double* wk[1] = {wmode};
  const double* sk[2] = {a->modes + 2 * NN, a->modes + 3 * NN};
  double* d = m->d_opws + 1024 * 16;
  HM_CHECK(dots(m, wk, 1, sk, 2, NN, d, m->d_opws));
  const double* wc[1] = {wmode + NN};
  const double* sc[1] = {a->modes + NN};
  HM_CHECK(dots(m, wc, 1, sc, 1, NN, d + 2, m->d_opws));
  hipLaunchKernelGGL(k_adr_final, dim3(1), dim3(64), 0, m->stream, out4, d, wmode + 2 * NN, theta[3]);
  HM_LAUNCH_CHECK();
  return HM_OK;
}

static void adr_release(Model* m) {
  AdrOp* a = (AdrOp*)m->op_ctx;
  if (!a) return;
  double* bufs[] = {a->E[0], a->E[1], a->W[0], a->W[1], a->lam[0], a->lam[1], a->mu, a->modes,
                    a->w[0], a->w[1], a->w[2], a->w[3], a->w[4]};
  for (double* p : bufs) dev_free(m->ctx, p);
  delete a;
  m->op_ctx = nullptr;
}

}  // namespace hm

using namespace hm;

extern "C" hm_status hm_model_create_adr(hm_ctx* ctx, int N, double kd, double vx, double vy, int leaf,
                                         hm_model** out) {
  if (!ctx || !out) {
    set_error("NULL argument");
    return HM_E_INVAL;
  }
  *out = nullptr;
  if (N < 2 || N > 1024 || !(kd > 0.0) || !std::isfinite(vx) || !std::isfinite(vy)) {
    set_error("hm_model_create_adr: need 2 <= N <= 1024, kd > 0, finite v");
    return HM_E_INVAL;
  }
  const double h = 1.0 / (N + 1);
  double rho[2], t[2];
  const double v[2] = {vx, vy};
  for (int a = 0; a < 2; ++a) {
    const double sub = -kd / (h * h) - v[a] / (2 * h), sup = -kd / (h * h) + v[a] / (2 * h);
    if (!(sub < 0.0 && sup < 0.0)) {
      set_error("hm_model_create_adr: the cell Peclet number |v| h / (2 kd) must be below 1");
      return HM_E_INVAL;
    }
    rho[a] = std::sqrt(sup / sub);
    t[a] = -std::sqrt(sub * sup);
    const double span = std::pow(rho[a], N - 1);
    if (span > 1e3 || span < 1e-3) {
      set_error("hm_model_create_adr: advection too strong for the similarity-transform solve "
                "(rho^(N-1) outside [1e-3, 1e3])");
      return HM_E_INVAL;
    }
  }
  // the grid points as coordinates (index y N + x): their KD-tree is the grid's bisection
  std::vector<double> xy((size_t)2 * N * N);
  for (int y = 0; y < N; ++y)
    for (int x = 0; x < N; ++x) {
      xy[2 * ((size_t)y * N + x)] = x;
      xy[2 * ((size_t)y * N + x) + 1] = y;
    }
  AdrOp* op = new AdrOp();
  op->N = N;
  hm_model* mm = nullptr;
  hm_status st = model_create_op(&ctx->c, 2, xy.data(), N * N, leaf, adr_apply, op, true, &mm);
  if (st != HM_OK) {
    delete op;
    return st;
  }
  Model* m = &mm->m;
  op->m = m;
  m->op_release = adr_release;
  m->op_vjp = adr_vjp;
  m->op_vjp_final = adr_vjp_final;
  // host tables
  const long NN = (long)N * N;
  std::vector<double> S((size_t)NN), E[2], W[2], lam[2], mu(N);
  for (int p = 0; p < N; ++p)
    for (int i = 0; i < N; ++i) S[(size_t)p + (size_t)i * N] = std::sqrt(2.0 / (N + 1)) * std::sin(M_PI * (p + 1) * (i + 1) / (N + 1));
  for (int p = 0; p < N; ++p) {
    const double s = std::sin(M_PI * (p + 1) / (2.0 * (N + 1)));
    mu[p] = 4.0 / (h * h) * s * s;
  }
  for (int a = 0; a < 2; ++a) {
    E[a].assign((size_t)NN, 0.0);
    W[a].assign((size_t)NN, 0.0);
    lam[a].resize(N);
    std::vector<double> d(N);
    for (int i = 0; i < N; ++i) d[i] = std::pow(rho[a], i);
    for (int p = 0; p < N; ++p) lam[a][p] = 2.0 * kd / (h * h) + 2.0 * t[a] * std::cos(M_PI * (p + 1) / (N + 1));
    for (int p = 0; p < N; ++p)
      for (int i = 0; i < N; ++i) E[a][(size_t)p + (size_t)i * N] = S[(size_t)p + (size_t)i * N] / d[i];   // S D^{-1}
    for (int p = 0; p < N; ++p)          // W = S D S (symmetric)
      for (int q = 0; q < N; ++q) {
        double acc = 0.0;
        for (int i = 0; i < N; ++i) acc += S[(size_t)p + (size_t)i * N] * d[i] * S[(size_t)i + (size_t)q * N];
        W[a][(size_t)p + (size_t)q * N] = acc;
      }
  }
  bool ok = true;
  auto A = [&](double** p, size_t doubles) {
    *p = (double*)dev_alloc(m->ctx, doubles * sizeof(double));
    ok = ok && *p;
  };
  for (int a = 0; a < 2; ++a) {
    A(&op->E[a], NN);
    A(&op->W[a], NN);
    A(&op->lam[a], N);
  }
  A(&op->mu, N);
  A(&op->modes, 4 * NN);
  for (int q = 0; q < 5; ++q) A(&op->w[q], (size_t)NN * m->cmax);
  if (!ok) {
    hm_model_destroy(mm);
    set_error("device allocation failed in hm_model_create_adr");
    return HM_E_NOMEM;
  }
  for (int a = 0; a < 2 && st == HM_OK; ++a) {
    if (hipMemcpy(op->E[a], E[a].data(), NN * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(op->W[a], W[a].data(), NN * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(op->lam[a], lam[a].data(), N * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
      st = HM_E_DEVICE;
  }
  if (st == HM_OK && hipMemcpy(op->mu, mu.data(), N * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
    st = HM_E_DEVICE;
  if (st != HM_OK) {
    hm_model_destroy(mm);
    set_error("hm_model_create_adr: copy of the tables failed");
    return st;
  }
  *out = mm;
  return HM_OK;
}
