// Bivariate co-kriging (two variables per grid node, the in-scope analogue of the
// bivariate model of Sec. 5.2, eq. "kphichi"; each block is the cov model of Sec. 2.1
// with the stencil operators of Sec. 5.1): one latent white noise w drives
//   y1 = sigma B^{-1} w + tau1 eps1,   y2 = sigma A^{-1} B^{-1} w + tau2 eps2,
//   K = sigma2 [[C, C A^{-T}], [A^{-1} C, A^{-1} C A^{-T}]] + diag(tau2_1 I, tau2_2 I),
// C = B^{-1} B^{-T}, theta_full = (kappa, alpha, tau2_1, sigma2, tau2_2), natural order
// y = (y1; y2).  The tree bisects the grid nodes and every node keeps its two rows
// together (variable 1 first).
//
// K-apply: A and B are diagonal in the orthonormal sine basis S (a = 1 + alpha mu,
// b = kappa^2 + mu per mode), so with u = S x1 + (S x2) / a,
//   K_op x = (S (u / b^2), S (u / (a b^2))):
// one forward transform of both halves, a per-mode combination, one inverse transform.
// The transforms are separable N x N products on the matrix cores (one GEMM along x
// over all columns, one batched GEMM along y).  Derivatives: d/dkappa replaces 1/b^2 by
// -4 kappa / b^3; d/dalpha differentiates r = 1/a (dr = -mu r^2):
//   y1 = (dr x2^) / b^2,   y2 = dr u / b^2 + r (dr x2^) / b^2   (in the sine basis).
#include <cmath>
#include <vector>

#include "hm_internal.h"
#include "gemm_core.h"

namespace hm {

struct BivOp {
  Model* m = nullptr;
  int dim = 2, N = 0;
  long NN = 0;
  double h = 0.0;
  double* S = nullptr;         // N x N orthonormal sine transform (symmetric)
  double* Ph = nullptr;        // N even: 2 x (H x H), Ph[par](q, i) = S(2q + par, i), H = N / 2
  double* mu = nullptr;        // NN eigenvalues of -Laplacian (x fastest)
  double* w[3] = {nullptr, nullptr, nullptr};   // NN x 2 cmax work buffers
};

// Folded transforms (N even, H = N / 2).  The sine transform's columns i and N-1-i
// differ by the sign (-1)^p of row p: S(p, N-1-i) = (-1)^p S(p, i).  So the rows of
// parity par of S X need only the H sums X(i) + (-1)^par X(N-1-i), i < H, and each
// pass is two H x H products instead of one N x N product.
struct BvHalfA {   // A(q, i) = Ph_par(q, i), q = m0 + row
  const double* p; int H, m0;
  static constexpr bool kfast = false;
  static constexpr int NR = 1;
  __device__ bool load(int i, int k, double (&v)[1]) const {
    const int r = m0 + i;
    const bool ok = r < H;
    v[0] = p[(ok ? r : 0) + (long)k * H];
    return ok;
  }
  __device__ double fin(const double (&v)[1]) const { return v[0]; }
};
struct BvFoldB {   // B(i, c) = X(i, c) + sgn X(N-1-i, c), X: N x R (ld N), c = n0 + col
  const double* X; int N; long n0, R; double sgn;
  static constexpr bool kfast = true;
  static constexpr int NR = 2;
  __device__ bool load(int k, int j, double (&v)[2]) const {
    const long c = n0 + j;
    const bool ok = c < R;
    const double* xc = X + (ok ? c : 0) * (long)N;
    v[0] = xc[k];
    v[1] = xc[N - 1 - k];
    return ok;
  }
  __device__ double fin(const double (&v)[2]) const { return v[0] + sgn * v[1]; }
};
struct BvStRows {   // Y(2 (m0 + i) + par, n0 + j), ld N
  double* Y; int N, H, m0; long n0, R; int par;
  __device__ void operator()(int i, int j, double v) const {
    const int r = m0 + i;
    const long c = n0 + j;
    if (r < H && c < R) Y[2 * r + par + c * N] = v;
  }
};
// Y = S X along the first axis: X, Y N x R (ld N).  grid.x: 2 ht (parity major), grid.y: R tiles
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k_biv_fold_rows(const double* Ph, const double* X, double* Y, int N, long R) {
  __shared__ double smem[GSMEM];
  const TileIdx tb = tile_block();
  const int H = N / 2, ht = (H + GBM - 1) / GBM;
  const int par = tb.x >= ht ? 1 : 0;
  const int m0 = (tb.x - par * ht) * GBM;
  const long n0 = (long)tb.y * GBN;
  TileAcc acc;
  tile_zero(acc);
  tile_gemm(BvHalfA{Ph + (long)par * H * H, H, m0}, BvFoldB{X, N, n0, R, par ? -1.0 : 1.0}, 0, H, acc, smem);
  tile_store(BvStRows{Y, N, H, m0, n0, R, par}, acc);
}
struct BvFoldA {   // A(p, y) = T(p, y) + sgn T(p, N-1-y), T: N x N (ld N)
  const double* T; int N, m0; double sgn;
  static constexpr bool kfast = false;
  static constexpr int NR = 2;
  __device__ bool load(int i, int k, double (&v)[2]) const {
    const int r = m0 + i;
    const bool ok = r < N;
    const int rr = ok ? r : 0;
    v[0] = T[rr + (long)k * N];
    v[1] = T[rr + (long)(N - 1 - k) * N];
    return ok;
  }
  __device__ double fin(const double (&v)[2]) const { return v[0] + sgn * v[1]; }
};
struct BvHalfB {   // B(y, q) = S(y, 2q + par) = Ph_par(q, y), q = n0 + col
  const double* p; int H, n0;
  static constexpr bool kfast = false;
  static constexpr int NR = 1;
  __device__ bool load(int k, int j, double (&v)[1]) const {
    const int c = n0 + j;
    const bool ok = c < H;
    v[0] = p[(ok ? c : 0) + (long)k * H];
    return ok;
  }
  __device__ double fin(const double (&v)[1]) const { return v[0]; }
};
struct BvStCols {   // Y(m0 + i, 2 (n0 + j) + par), ld N
  double* Y; int N, H, m0, n0, par;
  __device__ void operator()(int i, int j, double v) const {
    const int r = m0 + i, c = n0 + j;
    if (r < N && c < H) Y[r + (long)(2 * c + par) * N] = v;
  }
};
// Y_z = T_z S along the second axis for every slice z (N x N, stride NN).
// grid.x: row tiles, grid.y: 2 ht (parity major), grid.z: slices
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k_biv_fold_cols(const double* Ph, const double* T, double* Y, int N, long NN) {
  __shared__ double smem[GSMEM];
  const TileIdx tb = tile_block();
  const int H = N / 2, ht = (H + GBN - 1) / GBN;
  const int par = tb.y >= ht ? 1 : 0;
  const int m0 = tb.x * GBM, n0 = (tb.y - par * ht) * GBN;
  TileAcc acc;
  tile_zero(acc);
  tile_gemm(BvFoldA{T + tb.z * NN, N, m0, par ? -1.0 : 1.0}, BvHalfB{Ph + (long)par * H * H, H, n0}, 0, H, acc,
            smem);
  tile_store(BvStCols{Y + tb.z * NN, N, H, m0, n0, par}, acc);
}

// Y (NN x c', ld NN) = (S (x) S) X in 2D, S X in 1D; tmp: NN x c'
static hm_status biv_transform(const BivOp* b, hipStream_t st, const double* X, double* Y, double* tmp, int cp) {
  const int N = b->N;
  if (b->Ph) {
    const int H = N / 2;
    const long R = (long)cp * (b->dim == 1 ? 1 : N);   // columns of the first-axis product
    double* first = b->dim == 1 ? Y : tmp;
    hipLaunchKernelGGL(k_biv_fold_rows, dim3(2 * ceil_div(H, GBM), ceil_div(R, GBN)), dim3(GCfg::NT), 0, st, b->Ph,
                       X, first, N, R);
    HM_LAUNCH_CHECK();
    if (b->dim == 1) return HM_OK;
    hipLaunchKernelGGL(k_biv_fold_cols, dim3(ceil_div(N, GBM), 2 * ceil_div(H, GBN), cp), dim3(GCfg::NT), 0, st,
                       b->Ph, tmp, Y, N, b->NN);
    HM_LAUNCH_CHECK();
    return HM_OK;
  }
  if (b->dim == 1) return gemm(st, false, false, N, cp, N, 1.0, b->S, N, 0, X, N, 0, 0.0, Y, N, 0, 1);
  HM_CHECK(gemm(st, false, false, N, N * cp, N, 1.0, b->S, N, 0, X, N, 0, 0.0, tmp, N, 0, 1));
  return gemm(st, false, false, N, N, N, 1.0, tmp, N, b->NN, b->S, N, 0, 0.0, Y, N, b->NN, cp);
}

// per mode e and column j (halves 2j, 2j+1 of the NN x 2c layout)
__global__ void k_biv_modes(double* Yh, const double* Xh, const double* mu, long NN, int c, double kappa, double alpha,
                            int which) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= NN * c) return;
  const long i = e % NN, j = e / NN;
  const double x1 = Xh[i + 2 * j * NN], x2 = Xh[i + (2 * j + 1) * NN];
  const double mv = mu[i];
  const double r = 1.0 / (1.0 + alpha * mv);
  const double bb = kappa * kappa + mv;
  const double ib2 = 1.0 / (bb * bb);
  const double u = x1 + r * x2;
  double y1, y2;
  if (which == 0) {
    y1 = ib2 * u;
    y2 = r * ib2 * u;
  } else if (which == 1) {
    const double d = -4.0 * kappa * ib2 / bb;
    y1 = d * u;
    y2 = r * d * u;
  } else {
    const double dr = -mv * r * r;
    const double t = ib2 * dr * x2;
    y1 = t;
    y2 = dr * ib2 * u + r * t;
  }
  Yh[i + 2 * j * NN] = y1;
  Yh[i + (2 * j + 1) * NN] = y2;
}

static int biv_apply(void* uctx, int which, const double* theta, const double* X, long long ldx, long long cc,
                     double* Y, long long ldy, void* stream) {
  BivOp* b = (BivOp*)uctx;
  hipStream_t st = (hipStream_t)stream;
  const int c = (int)cc;
  if (!(theta[0] > 0.0) || !(theta[1] >= 0.0)) {
    set_error("theta must satisfy kappa > 0, alpha >= 0, tau2_1 > 0, sigma2 > 0, tau2_2 > 0");
    return HM_E_INVAL;
  }
  if (ldx != 2 * b->NN || ldy != 2 * b->NN || c > b->m->cmax || which < 0 || which > 2) {
    set_error("bivariate operator: unexpected block shape");
    return HM_E_INVAL;
  }
  // a column (x1; x2) of X is two consecutive NN-vectors: X is NN x 2c with ld NN
  HM_CHECK(biv_transform(b, st, X, b->w[0], b->w[2], 2 * c));
  hipLaunchKernelGGL(k_biv_modes, dim3(ceil_div(b->NN * c, 256)), dim3(256), 0, st, b->w[1], b->w[0], b->mu, b->NN, c,
                     theta[0], theta[1], which);
  HM_LAUNCH_CHECK();
  return biv_transform(b, st, b->w[1], Y, b->w[2], 2 * c);
}

static void biv_release(Model* m) {
  BivOp* b = (BivOp*)m->op_ctx;
  if (!b) return;
  double* bufs[] = {b->S, b->Ph, b->mu, b->w[0], b->w[1], b->w[2]};
  for (double* p : bufs) dev_free(m->ctx, p);
  delete b;
  m->op_ctx = nullptr;
}

hm_status model_create_bivariate(Ctx* cx, int dim, int N, double h, int leaf, hm_model** out) {
  if ((dim != 1 && dim != 2) || N < 2 || (dim == 2 && N > 4096) || !(h > 0.0) || !std::isfinite(h)) {
    set_error("bivariate model: need dim in {1,2}, N >= 2 (2D: N <= 4096), h > 0");
    return HM_E_INVAL;
  }
  const long NN = (long)N * (dim == 2 ? N : 1);
  std::vector<double> xy((size_t)NN * dim);
  for (long g = 0; g < NN; ++g) {
    if (dim == 2) {
      xy[2 * g] = (double)(g % N);
      xy[2 * g + 1] = (double)(g / N);
    } else {
      xy[g] = (double)g;
    }
  }
  BivOp* b = new BivOp();
  b->dim = dim;
  b->N = N;
  b->NN = NN;
  b->h = h;
  hm_model* mm = nullptr;
  hm_status st = model_create_op(cx, dim, xy.data(), (int)NN, leaf, biv_apply, b, true, &mm, 2);
  if (st != HM_OK) {
    delete b;
    return st;
  }
  Model* m = &mm->m;
  b->m = m;
  m->op_release = biv_release;
  // host tables: S and the modes' eigenvalues of -Laplacian (x fastest)
  std::vector<double> S((size_t)N * N), mu1(N), mu((size_t)NN);
  const double sc = std::sqrt(2.0 / (N + 1));
  for (int p = 0; p < N; ++p)
    for (int i = 0; i < N; ++i) S[(size_t)p + (size_t)i * N] = sc * std::sin(M_PI * (p + 1.0) * (i + 1.0) / (N + 1));
  for (int p = 0; p < N; ++p) {
    const double s = std::sin(M_PI * (p + 1.0) / (2.0 * (N + 1)));
    mu1[p] = 4.0 / (h * h) * s * s;
  }
  for (long e = 0; e < NN; ++e) mu[e] = dim == 2 ? mu1[e % N] + mu1[e / N] : mu1[e];
  bool ok = true;
  auto A = [&](double** p, size_t doubles) {
    *p = (double*)dev_alloc(m->ctx, doubles * sizeof(double));
    ok = ok && *p;
  };
  A(&b->S, (size_t)N * N);
  const int H = N / 2;
  if (N % 2 == 0) A(&b->Ph, (size_t)2 * H * H);
  A(&b->mu, (size_t)NN);
  for (int q = 0; q < 3; ++q) A(&b->w[q], (size_t)NN * 2 * m->cmax);
  if (!ok) {
    hm_model_destroy(mm);
    set_error("device allocation failed in the bivariate model");
    return HM_E_NOMEM;
  }
  std::vector<double> Ph(b->Ph ? (size_t)2 * H * H : 0);
  for (int par = 0; par < 2 && b->Ph; ++par)
    for (int q = 0; q < H; ++q)
      for (int i = 0; i < H; ++i) Ph[(size_t)par * H * H + q + (size_t)i * H] = S[(size_t)(2 * q + par) + (size_t)i * N];
  if ((b->Ph && hipMemcpy(b->Ph, Ph.data(), Ph.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) ||
      hipMemcpy(b->S, S.data(), S.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->mu, mu.data(), mu.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
    hm_model_destroy(mm);
    set_error("bivariate model: copy of the tables failed");
    return HM_E_DEVICE;
  }
  *out = mm;
  return HM_OK;
}

}  // namespace hm
