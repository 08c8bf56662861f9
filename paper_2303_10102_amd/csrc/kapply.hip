// Physics K-apply: Y = K X, dK/dkappa X, dK/dalpha X for blocks of vectors.
//
// K = sigma2 A^{-1} B^{-1} B^{-T} A^{-T} + tau2 I with B = kappa^2 I + T, A = I + alpha T,
// T = -Lap (Dirichlet, h = 1/(N+1)).  The paper accesses K only through such
// products (Sec. 3.2) and its derivatives by differentiating them (Sec. 3.3).
// The solves are exact and direct (a fast Poisson-type solver): the orthonormal
// DST-I along x and along y diagonalises the constant-coefficient Dirichlet
// stencils, so A^{-1}, B^{-1} and their parameter derivatives become per-mode
// scalings by
//   e(p,q)      = sigma2 / ((1 + alpha mu)^2 (kappa^2 + mu)^2) + tau2,   mu = mu_p + mu_q
//   de/dkappa   = -4 kappa lam / (kappa^2 + mu),   de/dalpha = -2 mu lam / (1 + alpha mu).
// Each transform is an N x N GEMM over all columns at once (tree<->grid
// permutation fused into the first load and the last store); the forward
// transforms are shared by the value and both tangents.  The H-matrix method
// never sees this structure: it only calls the products.
#include <cmath>

#include "gemm_core.h"
#include "hm_internal.h"

namespace hm {

// ---------------------------------------------------------------------------
// tree ordering (recursive coordinate bisection, uniform splits) and tables
// ---------------------------------------------------------------------------
__global__ void k_perm(int* perm, int* iperm, int n, int N, int dim, int levels, int nl) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  int L = t / nl, q = t % nl;
  int x0 = 0, y0 = 0, w = N, h = (dim == 2) ? N : 1;
  for (int d = levels - 1; d >= 0; --d) {
    int bit = (L >> d) & 1;
    if (w >= h) {
      int wl = w / 2;
      if (bit) { x0 += wl; w -= wl; } else { w = wl; }
    } else {
      int hl = h / 2;
      if (bit) { y0 += hl; h -= hl; } else { h = hl; }
    }
  }
  int x = x0 + q % w, y = y0 + q / w;
  int g = (dim == 2) ? y * N + x : x;
  perm[t] = g;
  iperm[g] = t;
}

__global__ void k_tables(double* S, double* mu, int N, int dim) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  const double scale = sqrt(2.0 / (N + 1));
  if (e < N * N) {
    int p = e % N, x = e / N;
    long m = (long)(p + 1) * (x + 1) % (2L * (N + 1));
    S[e] = scale * sinpi((double)m / (double)(N + 1));
  }
  if (e < N) {
    const double h = 1.0 / (N + 1);
    double s = sinpi((double)(e + 1) / (2.0 * (N + 1)));
    mu[e] = 4.0 / (h * h) * s * s;
  }
}

// Per-mode multipliers for K, dK/dkappa, dK/dalpha: lam[o*N*Ny + p + q*N]
__global__ void k_mode_scale(double* lam, const double* mu, int N, int Ny, double kappa, double alpha,
                             double tau2, double sigma2) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * Ny) return;
  int p = e % N, q = e / N;
  double m = mu[p] + (Ny > 1 ? mu[q] : 0.0);
  double a = 1.0 + alpha * m, b = kappa * kappa + m;
  double l = sigma2 / (a * a * b * b);
  const long NN = (long)N * Ny;
  lam[e] = l + tau2;
  lam[NN + e] = -4.0 * kappa * l / b;
  lam[2 * NN + e] = -2.0 * m * l / a;
}

// ---------------------------------------------------------------------------
// sine transforms with fused tree<->grid permutation
//
// Axis maps.  A sketch pass at depth l reads an input that is zero outside one
// side (left or right children) of the depth-l split and needs the output only on
// the other side; both sides are alternating chunks of width W along the split
// axis.  AxisMap{W, par} enumerates the coordinates t -> (t / W) 2W + par W + t % W
// (the chunks of parity par); W = 0 is the whole axis.  The transforms then run
// over the compact half: the forward x-transform sums only the input's x, the
// y-transforms only the input's / needed y, the inverse x-transform writes only
// the needed x.
// ---------------------------------------------------------------------------
struct AxisMap {
  int W, par;
  __host__ __device__ int operator()(int t) const { return W ? (t / W) * 2 * W + par * W + t % W : t; }
  __host__ __device__ int extent(int n) const { return W ? n / 2 : n; }
};

// Column r of a transform operand is (col, y') = (r / Ny, r % Ny) over the compact
// y range Ny.  AM: 0 general division, 1 a tile of GBN columns lies inside one
// grid column (Ny % GBN == 0), 2 one-dimensional (Ny == 1).
template <int AM>
__device__ __forceinline__ void split_col(int r, int Ny, int colt, int yt, int j, int& col, int& y) {
  if (AM == 2) { col = r; y = 0; }
  else if (AM == 1) { col = colt; y = yt + j; }
  else { col = r / Ny; y = r - col * Ny; }
}
struct DstLS {  // A(i, k) = S(m0 + i, xmap(k))   (S symmetric, N x N)
  const double* S; int N, m0; AxisMap xm;
  static constexpr bool kfast = false;
  __device__ double operator()(int i, int k) const {
    int p = m0 + i;
    return p < N ? S[p + (long)xm(k) * N] : 0.0;
  }
};
struct DstLSrow {  // A(i, k) = S(xmap(m0 + i), k) for i < Mx
  const double* S; int N, m0, Mx; AxisMap xm;
  static constexpr bool kfast = false;
  __device__ double operator()(int i, int k) const {
    int r = m0 + i;
    return r < Mx ? S[xm(r) + (long)k * N] : 0.0;
  }
};
template <int AM>
struct DstLGather {  // B(k, j) = X[col*ldx + iperm[ymap(y')*N + xmap(k)]]
  const double* X; int ldx; const int* iperm; int N, Ny, n0, R, colt, yt; AxisMap xm, ym;
  static constexpr bool kfast = true;
  __device__ double operator()(int k, int j) const {
    int r = n0 + j;
    if (r >= R) return 0.0;
    int col, y;
    split_col<AM>(r, Ny, colt, yt, j, col, y);
    return X[(long)col * ldx + iperm[ym(y) * N + xm(k)]];
  }
};
template <int AM>
struct DstLMode {  // B(p, r) = W[p + r*N] (optionally scaled by lam[p + ymap(y')*N], 1D: lam[p])
  const double* W; const double* lam; int N, Ny, n0, R, colt, yt; AxisMap ym;
  static constexpr bool kfast = true;
  __device__ double operator()(int k, int j) const {
    int r = n0 + j;
    if (r >= R) return 0.0;
    double v = W[k + (long)r * N];
    if (lam) {
      int col, y;
      split_col<AM>(r, Ny, colt, yt, j, col, y);
      v *= lam[k + (long)ym(y) * N];
    }
    return v;
  }
};
struct DstStMode {
  double* p; int N, m0, n0, R;
  __device__ void operator()(int i, int j, double v) const {
    int pp = m0 + i, r = n0 + j;
    if (pp < N && r < R) p[pp + (long)r * N] = v;
  }
};
template <int AM>
struct DstStScatter {  // Y[col*ldy + iperm[ymap(y')*N + xmap(i)]]
  double* Y; int ldy; const int* iperm; int N, Ny, m0, n0, Mx, R, colt, yt; AxisMap xm, ym;
  __device__ void operator()(int i, int j, double v) const {
    int xi = m0 + i, r = n0 + j;
    if (xi >= Mx || r >= R) return;
    int col, y;
    split_col<AM>(r, Ny, colt, yt, j, col, y);
    Y[(long)col * ldy + iperm[ym(y) * N + xm(xi)]] = v;
  }
};
// y-direction transforms of every column's N x Nyin block M (rows p, cols y'):
//   forward  C_c(p, q)  = sum_{y'} M_c(p, y') S(ymap(y'), q)          (Nyin compact, q full)
//   inverse  C_c(p, y') = sum_q (lam o M_c)(p, q) S(q, ymap(y'))      (q full, y' compact)
struct DyLA {
  const double* M; const double* lam; int N, m0;
  static constexpr bool kfast = false;
  __device__ double operator()(int i, int k) const {
    int p = m0 + i;
    if (p >= N) return 0.0;
    double v = M[p + (long)k * N];
    if (lam) v *= lam[p + (long)k * N];
    return v;
  }
};
struct DyLBfwd {  // B(k, j) = S(ymap(k), n0 + j)
  const double* S; int N, n0; AxisMap ym;
  static constexpr bool kfast = true;
  __device__ double operator()(int k, int j) const {
    int q = n0 + j;
    return q < N ? S[ym(k) + (long)q * N] : 0.0;
  }
};
struct DyLBinv {  // B(k, j) = S(k, ymap(n0 + j)) for j < Nout
  const double* S; int N, n0, Nout; AxisMap ym;
  static constexpr bool kfast = true;
  __device__ double operator()(int k, int j) const {
    int c = n0 + j;
    return c < Nout ? S[k + (long)ym(c) * N] : 0.0;
  }
};

// Xh(p, r) = sum_{x'} S(p, xmap(x')) X[col*ldx + iperm[ymap(y')*N + xmap(x')]],  r = col*Ny + y'
template <int AM>
__global__ void __launch_bounds__(256) k_dst_fwd(const double* S, const double* X, int ldx, const int* iperm,
                                                 double* Xh, int N, int Ny, int ncol, int Kx, AxisMap xm,
                                                 AxisMap ym) {
  __shared__ double smem[GSMEM];
  const int m0 = blockIdx.x * GBM, n0 = blockIdx.y * GBN;
  const int R = ncol * Ny;
  const int colt = (AM == 1) ? n0 / Ny : 0, yt = (AM == 1) ? n0 - colt * Ny : 0;
  DstLS la{S, N, m0, xm};
  DstLGather<AM> lb{X, ldx, iperm, N, Ny, n0, R, colt, yt, xm, ym};
  TileAcc acc;
  tile_zero(acc);
  tile_gemm(la, lb, 0, Kx, acc, smem);
  DstStMode st{Xh, N, m0, n0, R};
  tile_store(st, acc);
}

// forward y: C_c = M_c S[ymap(.), :]  (M_c: N x Nyin at c*N*Nyin; C_c: N x N at c*N*N)
__global__ void __launch_bounds__(256) k_dst_yf(const double* S, const double* M, double* C, int N, int Nyin,
                                                AxisMap ym) {
  __shared__ double smem[GSMEM];
  const int m0 = blockIdx.x * GBM, n0 = blockIdx.y * GBN;
  DyLA la{M + (long)blockIdx.z * N * Nyin, nullptr, N, m0};
  DyLBfwd lb{S, N, n0, ym};
  TileAcc acc;
  tile_zero(acc);
  tile_gemm(la, lb, 0, Nyin, acc, smem);
  DstStMode st{C + (long)blockIdx.z * N * N, N, m0, n0, N};
  tile_store(st, acc);
}

// inverse y: C_c = (lam o M_c) S[:, ymap(.)]  (M_c: N x N; C_c: N x Nyout at c*N*Nyout)
__global__ void __launch_bounds__(256) k_dst_yi(const double* S, const double* M, const double* lam, double* C,
                                                int N, int Nyout, AxisMap ym) {
  __shared__ double smem[GSMEM];
  const int m0 = blockIdx.x * GBM, n0 = blockIdx.y * GBN;
  DyLA la{M + (long)blockIdx.z * N * N, lam, N, m0};
  DyLBinv lb{S, N, n0, Nyout, ym};
  TileAcc acc;
  tile_zero(acc);
  tile_gemm(la, lb, 0, N, acc, smem);
  DstStMode st{C + (long)blockIdx.z * N * Nyout, N, m0, n0, Nyout};
  tile_store(st, acc);
}

// Y[col*ldy + iperm[ymap(y')*N + xmap(x')]] = sum_p S(xmap(x'), p) (lam o W)(p, r)
template <int AM>
__global__ void __launch_bounds__(256) k_dst_inv(const double* S, const double* W, const double* lam,
                                                 const int* iperm, double* Y, int ldy, int N, int Ny, int ncol,
                                                 int Mx, AxisMap xm, AxisMap ym) {
  __shared__ double smem[GSMEM];
  const int m0 = blockIdx.x * GBM, n0 = blockIdx.y * GBN;
  const int R = ncol * Ny;
  const int colt = (AM == 1) ? n0 / Ny : 0, yt = (AM == 1) ? n0 - colt * Ny : 0;
  DstLSrow la{S, N, m0, Mx, xm};
  DstLMode<AM> lb{W, lam, N, Ny, n0, R, colt, yt, ym};
  TileAcc acc;
  tile_zero(acc);
  tile_gemm(la, lb, 0, N, acc, smem);
  DstStScatter<AM> st{Y, ldy, iperm, N, Ny, m0, n0, Mx, R, colt, yt, xm, ym};
  tile_store(st, acc);
}

static hm_status ensure_scale(Model* m, const double theta[4]) {
  bool same = true;
  for (int i = 0; i < 4; ++i) same = same && (m->lam_key[i] == theta[i]);
  if (same) return HM_OK;
  const int Ny = (m->dim == 2) ? m->N : 1;
  hipLaunchKernelGGL(k_mode_scale, dim3(ceil_div((long)m->N * Ny, 256)), dim3(256), 0, m->stream, m->d_lam,
                     m->d_mu, m->N, Ny, theta[0], theta[1], theta[2], theta[3]);
  HM_LAUNCH_CHECK();
  for (int i = 0; i < 4; ++i) m->lam_key[i] = theta[i];
  return HM_OK;
}

// Axis map of the rows selected by sel (one side of the depth-sel.depth split):
// simulate the bisection to find the split axis and the children's extent on it.
static void side_maps(const Model* m, LeafSel sel, AxisMap& xm, AxisMap& ym) {
  xm = AxisMap{0, 0};
  ym = AxisMap{0, 0};
  if (sel.mode == 0) return;
  int w = m->N, h = (m->dim == 2) ? m->N : 1;
  bool xsplit = true;
  for (int d = 1; d <= sel.depth; ++d) {
    if (w >= h) { w /= 2; xsplit = true; }
    else { h /= 2; xsplit = false; }
  }
  const AxisMap am{xsplit ? w : h, sel.mode == 2 ? 1 : 0};
  if (xsplit) xm = am;
  else ym = am;
}

template <int AM>
static void launch_fwd(Model* m, dim3 g, const double* X, int ldx, double* out, int N, int Ny, int cc, int Kx,
                       AxisMap xm, AxisMap ym) {
  hipLaunchKernelGGL((k_dst_fwd<AM>), g, dim3(GCfg::NT), 0, m->stream, m->d_dst, X, ldx, m->d_iperm, out, N, Ny,
                     cc, Kx, xm, ym);
}
template <int AM>
static void launch_inv(Model* m, dim3 g, const double* W, const double* lam, double* Y, int ldy, int N, int Ny,
                       int cc, int Mx, AxisMap xm, AxisMap ym) {
  hipLaunchKernelGGL((k_dst_inv<AM>), g, dim3(GCfg::NT), 0, m->stream, m->d_dst, W, lam, m->d_iperm, Y, ldy, N, Ny,
                     cc, Mx, xm, ym);
}

hm_status kapply_sel(Model* m, const double theta[4], const double* X, int ldx, int c, double* outK,
                     double* outKap, double* outAlp, int ldo, LeafSel in_sel, LeafSel out_sel) {
  if (c <= 0) return HM_OK;
  HM_CHECK(ensure_scale(m, theta));
  const int n = m->n, N = m->N;
  const bool two = (m->dim == 2);
  const int Nyf = two ? N : 1;
  const long NN = (long)N * Nyf;
  AxisMap xin, yin, xout, yout;
  side_maps(m, in_sel, xin, yin);
  side_maps(m, out_sel, xout, yout);
  const int Kx = xin.extent(N), Mx = xout.extent(N);
  const int Nyi = two ? yin.extent(N) : 1, Nyo = two ? yout.extent(N) : 1;
  double* Xh = m->d_ws;                        // x-transformed (compact input y)
  double* X2 = m->d_ws + (long)n * m->cmax;    // x- and y-transformed (2D)
  double* X3 = m->d_ws + 2L * n * m->cmax;     // scaled and y-inverse-transformed (compact output y)
  double* outs[3] = {outK, outKap, outAlp};
  const bool pf = prof_on(m, PF_DST);
  int nout = 0;
  for (int q = 0; q < 3; ++q) nout += outs[q] ? 1 : 0;
  // algorithmic work of the transform GEMMs actually run, per column
  const double fl_fwd = 2.0 * N * Kx * Nyi + (two ? 2.0 * N * Nyi * (double)N : 0.0);
  const double fl_out = (two ? 2.0 * N * N * (double)Nyo : 0.0) + 2.0 * Mx * N * (double)Nyo;
  const double per_col = fl_fwd + nout * fl_out;
  if (pf) prof_begin(m, PF_DST);
  auto amode = [](int ny) { return ny == 1 ? 2 : (ny % GBN == 0 ? 1 : 0); };
  for (int c0 = 0; c0 < c; c0 += m->cmax) {
    const int cc = std::min(m->cmax, c - c0);
    const double* Xc = X + (long)c0 * ldx;
    dim3 gx(ceil_div(N, GBM), ceil_div((long)cc * Nyi, GBN));
    const int ami = amode(Nyi);
    if (ami == 2) launch_fwd<2>(m, gx, Xc, ldx, Xh, N, Nyi, cc, Kx, xin, yin);
    else if (ami == 1) launch_fwd<1>(m, gx, Xc, ldx, Xh, N, Nyi, cc, Kx, xin, yin);
    else launch_fwd<0>(m, gx, Xc, ldx, Xh, N, Nyi, cc, Kx, xin, yin);
    HM_LAUNCH_CHECK();
    if (two) {
      dim3 gy(ceil_div(N, GBM), ceil_div(N, GBN), cc);
      hipLaunchKernelGGL(k_dst_yf, gy, dim3(GCfg::NT), 0, m->stream, m->d_dst, Xh, X2, N, Nyi, yin);
      HM_LAUNCH_CHECK();
    }
    const int amo = amode(Nyo);
    for (int q = 0; q < 3; ++q) {
      if (!outs[q]) continue;
      const double* lam = m->d_lam + q * NN;
      double* Yc = outs[q] + (long)c0 * ldo;
      dim3 gi(ceil_div(Mx, GBM), ceil_div((long)cc * Nyo, GBN));
      if (two) {
        dim3 gy(ceil_div(N, GBM), ceil_div(Nyo, GBN), cc);
        hipLaunchKernelGGL(k_dst_yi, gy, dim3(GCfg::NT), 0, m->stream, m->d_dst, X2, lam, X3, N, Nyo, yout);
        HM_LAUNCH_CHECK();
        if (amo == 1) launch_inv<1>(m, gi, X3, nullptr, Yc, ldo, N, Nyo, cc, Mx, xout, yout);
        else launch_inv<0>(m, gi, X3, nullptr, Yc, ldo, N, Nyo, cc, Mx, xout, yout);
      } else {
        launch_inv<2>(m, gi, Xh, lam, Yc, ldo, N, 1, cc, Mx, xout, yout);
      }
      HM_LAUNCH_CHECK();
    }
  }
  if (pf) {
    // bytes: each pass reads and writes its n x c block once (compact where the maps halve it), plus S
    const double frac_in = (double)Kx * Nyi / NN, frac_out = (double)Mx * Nyo / NN;
    const double passes = (two ? 1.0 + 1.0 : 1.0) * (0.5 + 0.5 * frac_in) + nout * (two ? 2.0 : 1.0) * 0.5 * (1.0 + frac_out);
    prof_end(m, PF_DST, per_col * c, passes * 16.0 * n * (double)c + 8.0 * N * (double)N);
  }
  return HM_OK;
}

hm_status kapply(Model* m, const double theta[4], const double* X, int ldx, int c, double* outK,
                 double* outKap, double* outAlp, int ldo) {
  return kapply_sel(m, theta, X, ldx, c, outK, outKap, outAlp, ldo, sel_all(), sel_all());
}

hm_status model_tables(Model* m) {
  const int n = m->n, N = m->N;
  hipLaunchKernelGGL(k_perm, dim3(ceil_div(n, 256)), dim3(256), 0, m->stream, m->d_perm, m->d_iperm, n, N,
                     m->dim, m->levels, m->nl);
  HM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_tables, dim3(ceil_div((long)N * N, 256)), dim3(256), 0, m->stream, m->d_dst, m->d_mu, N,
                     m->dim);
  HM_LAUNCH_CHECK();
  return HM_OK;
}

}  // namespace hm

namespace hm {

// wmode[m] += sum_c (S P X)[m, c] (S P Ybar)[m, c]: the per-mode weights of the
// K-apply's vector-Jacobian product.  For Y = K(theta) X (X independent of theta),
//   <Ybar, dK/dtheta_j X> = sum_m de_m/dtheta_j * wmode[m],
// since every operator of the family is P^T S diag(.) S P with the same S.
__global__ void k_mode_dot(const double* A, const double* B, long NN, int cc, double* wmode) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= NN) return;
  double s = 0.0;
  for (int c = 0; c < cc; ++c) s += A[e + c * NN] * B[e + c * NN];
  wmode[e] += s;
}

hm_status kvjp(Model* m, const double theta[4], const double* X, int ldx, const double* Yb, int ldb, int c,
               double* wmode) {
  if (c <= 0) return HM_OK;
  HM_CHECK(ensure_scale(m, theta));
  const int n = m->n, N = m->N;
  const int Ny = (m->dim == 2) ? N : 1;
  const long NN = (long)N * Ny;
  double* W0 = m->d_ws;
  double* W1 = m->d_ws + (long)n * m->cmax;
  double* W2 = m->d_ws + 2L * n * m->cmax;
  const int am = (Ny == 1) ? 2 : (Ny % GBN == 0 ? 1 : 0);
  const AxisMap id{0, 0};
  for (int c0 = 0; c0 < c; c0 += m->cmax) {
    const int cc = std::min(m->cmax, c - c0);
    dim3 gx(ceil_div(N, GBM), ceil_div((long)cc * Ny, GBN));
    dim3 gy(ceil_div(N, GBM), ceil_div(N, GBN), cc);
    const double* Xc = X + (long)c0 * ldx;
    const double* Bc = Yb + (long)c0 * ldb;
    const double *ha, *hb;
    auto fwd = [&](const double* src, int ld, double* dst) {
      if (am == 2) launch_fwd<2>(m, gx, src, ld, dst, N, Ny, cc, N, id, id);
      else if (am == 1) launch_fwd<1>(m, gx, src, ld, dst, N, Ny, cc, N, id, id);
      else launch_fwd<0>(m, gx, src, ld, dst, N, Ny, cc, N, id, id);
    };
    if (m->dim == 2) {
      fwd(Xc, ldx, W0);
      HM_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_dst_yf, gy, dim3(GCfg::NT), 0, m->stream, m->d_dst, W0, W1, N, N, id);
      HM_LAUNCH_CHECK();
      fwd(Bc, ldb, W2);
      HM_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_dst_yf, gy, dim3(GCfg::NT), 0, m->stream, m->d_dst, W2, W0, N, N, id);
      HM_LAUNCH_CHECK();
      ha = W1;
      hb = W0;
    } else {
      fwd(Xc, ldx, W0);
      HM_LAUNCH_CHECK();
      fwd(Bc, ldb, W1);
      HM_LAUNCH_CHECK();
      ha = W0;
      hb = W1;
    }
    hipLaunchKernelGGL(k_mode_dot, dim3(ceil_div(NN, 256)), dim3(256), 0, m->stream, ha, hb, NN, cc, wmode);
    HM_LAUNCH_CHECK();
  }
  return HM_OK;
}

}  // namespace hm
