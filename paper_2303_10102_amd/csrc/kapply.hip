// Physics K-apply: Y = K X, dK/dkappa X, dK/dalpha X for blocks of vectors.
//
// K = sigma2 A^{-1} B^{-1} B^{-T} A^{-T} + tau2 I with B = kappa^2 I + T, A = I + alpha T,
// T = -Lap (Dirichlet, h = 1/(N+1)); A and B are symmetric.  The paper accesses K
// only through such products (Sec. 3.2) and its derivatives by forward-mode
// differentiation of the solves (Sec. 3.3).  The solves are exact and direct:
//   2D: orthonormal DST-I along x (an N x N GEMM over all columns at once, the
//       tree->grid gather fused into its operand load), then for every x-mode p a
//       chain of tridiagonal solves along y with A_p = (1+alpha mu_p) I + alpha T_y,
//       B_p = (kappa^2 + mu_p) I + T_y, then the inverse DST with the grid->tree
//       scatter fused into its store.
//   1D: the same chain on the single line (mu = 0).
// The tangent chains share the forward transform and the value chain's
// intermediates (forward-mode AD of the solve sequence).
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
  if (dim == 2 && e < N * N) {
    int p = e % N, x = e / N;
    long m = (long)(p + 1) * (x + 1) % (2L * (N + 1));
    S[e] = scale * sinpi((double)m / (double)(N + 1));
  }
  if (e < N) {
    const double h = 1.0 / (N + 1);
    double s = sinpi((double)(e + 1) / (2.0 * (N + 1)));
    mu[e] = (dim == 2) ? 4.0 / (h * h) * s * s : 0.0;
  }
}

// LU (Thomas) coefficients of A_p and B_p, layout [i*Np + p]
__global__ void k_thomas_coef(double* coef, const double* mu, int L, int Np, double kappa, double alpha,
                              double h2inv) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= Np) return;
  double* cA = coef;
  double* imA = coef + (long)L * Np;
  double* cB = coef + 2L * L * Np;
  double* imB = coef + 3L * L * Np;
  const double dA = 1.0 + alpha * mu[p] + 2.0 * alpha * h2inv, eA = -alpha * h2inv;
  const double dB = kappa * kappa + mu[p] + 2.0 * h2inv, eB = -h2inv;
  double ca = 0.0, cb = 0.0;
  for (int i = 0; i < L; ++i) {
    double ma = dA - eA * ca, mb = dB - eB * cb;
    ca = eA / ma;
    cb = eB / mb;
    cA[(long)i * Np + p] = ca;
    imA[(long)i * Np + p] = 1.0 / ma;
    cB[(long)i * Np + p] = cb;
    imB[(long)i * Np + p] = 1.0 / mb;
  }
}

// ---------------------------------------------------------------------------
// tridiagonal chains along a line: element i at w[i*s]
// ---------------------------------------------------------------------------
struct Line {
  const double* c;   // c_i at c[i*Np]
  const double* im;  // 1/m_i
  double e;          // off-diagonal
};

__device__ __forceinline__ void tri_solve(double* w, long s, int L, const Line& op, int Np) {
  double prev = 0.0;
  for (int i = 0; i < L; ++i) {
    double v = (w[i * s] - op.e * prev) * op.im[(long)i * Np];
    w[i * s] = v;
    prev = v;
  }
  double nxt = w[(long)(L - 1) * s];
  for (int i = L - 2; i >= 0; --i) {
    double v = w[i * s] - op.c[(long)i * Np] * nxt;
    w[i * s] = v;
    nxt = v;
  }
}

// dst = a*dst + b * (dA src), dA = mu I + T_y (T_y = h2inv * tridiag(-1,2,-1))
__device__ __forceinline__ void apply_dA(double* dst, const double* src, long s, int L, double mu,
                                         double h2inv, double a, double b) {
  double left = 0.0, cur = src[0];
  for (int i = 0; i < L; ++i) {
    double right = (i + 1 < L) ? src[(i + 1) * s] : 0.0;
    double v = mu * cur + h2inv * (2.0 * cur - left - right);
    dst[i * s] = (a == 0.0 ? 0.0 : a * dst[i * s]) + b * v;
    left = cur;
    cur = right;
  }
}

template <int MODE>  // bit0 value K, bit1 d/dkappa, bit2 d/dalpha
__global__ void k_thomas_chain(const double* __restrict__ U, double* W, double* Tk, double* Ta, int ncol,
                               int n, int L, int Np, const double* coef, const double* mu, double kappa,
                               double alpha, double sigma2, double tau2, double h2inv) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ncol * Np) return;
  const int col = t / Np, p = t % Np;
  const long base = (long)col * n + p;
  const long s = Np;
  Line A{coef + p, coef + (long)L * Np + p, -alpha * h2inv};
  Line B{coef + 2L * L * Np + p, coef + 3L * L * Np + p, -h2inv};
  const double mup = mu[p];
  double* w = W + base;
  double* tk = (MODE & 2) ? Tk + base : nullptr;
  double* ta = (MODE & 4) ? Ta + base : nullptr;
  const double* u = U + base;
  for (int i = 0; i < L; ++i) w[i * s] = u[i * s];
  tri_solve(w, s, L, A, Np);                                       // v1 = A^-1 u
  if (MODE & 4) {
    apply_dA(ta, w, s, L, mup, h2inv, 0.0, -1.0);                   // -dA v1
    tri_solve(ta, s, L, A, Np);                                     // t1 = -A^-1 dA v1
  }
  tri_solve(w, s, L, B, Np);                                       // v2 = B^-1 v1
  if (MODE & 2) {
    for (int i = 0; i < L; ++i) tk[i * s] = -2.0 * kappa * w[i * s];
    tri_solve(tk, s, L, B, Np);                                     // t2 = -2k B^-1 v2
  }
  if (MODE & 4) tri_solve(ta, s, L, B, Np);                        // t2 = B^-1 t1
  tri_solve(w, s, L, B, Np);                                       // v3 = B^-1 v2
  if (MODE & 2) {
    for (int i = 0; i < L; ++i) tk[i * s] -= 2.0 * kappa * w[i * s];
    tri_solve(tk, s, L, B, Np);                                     // t3 = B^-1 (t2 - 2k v3)
    tri_solve(tk, s, L, A, Np);                                     // t4 = A^-1 t3
  }
  if (MODE & 4) tri_solve(ta, s, L, B, Np);                        // t3 = B^-1 t2
  tri_solve(w, s, L, A, Np);                                       // v4 = A^-1 v3
  if (MODE & 4) {
    apply_dA(ta, w, s, L, mup, h2inv, 1.0, -1.0);                   // t3 - dA v4
    tri_solve(ta, s, L, A, Np);                                     // t4
  }
  if (MODE & 1)
    for (int i = 0; i < L; ++i) w[i * s] = sigma2 * w[i * s] + tau2 * u[i * s];
  if (MODE & 2)
    for (int i = 0; i < L; ++i) tk[i * s] *= sigma2;
  if (MODE & 4)
    for (int i = 0; i < L; ++i) ta[i * s] *= sigma2;
}

// ---------------------------------------------------------------------------
// sine transforms with fused tree<->grid permutation (2D)
// ---------------------------------------------------------------------------
struct DstLS {  // S (N x N, symmetric), rows m0..
  const double* S; int N, m0;
  static constexpr bool kfast = false;
  __device__ double operator()(int i, int k) const {
    int p = m0 + i;
    return p < N ? S[p + (long)k * N] : 0.0;
  }
};
struct DstLGather {  // B(x, r) = X[col*ldx + iperm[y*N + x]],  r = col*N + y
  const double* X; int ldx; const int* iperm; int N, n0, R;
  static constexpr bool kfast = true;
  __device__ double operator()(int k, int j) const {
    int r = n0 + j;
    if (r >= R) return 0.0;
    int col = r / N, y = r - col * N;
    return X[(long)col * ldx + iperm[y * N + k]];
  }
};
struct DstLMode {  // B(p, r) = W[p + r*N]
  const double* W; int N, n0, R;
  static constexpr bool kfast = true;
  __device__ double operator()(int k, int j) const {
    int r = n0 + j;
    return r < R ? W[k + (long)r * N] : 0.0;
  }
};
struct DstStMode {
  double* p; int N, m0, n0, R;
  __device__ void operator()(int i, int j, double v) const {
    int pp = m0 + i, r = n0 + j;
    if (pp < N && r < R) p[pp + (long)r * N] = v;
  }
};
struct DstStScatter {
  double* Y; int ldy; const int* iperm; int N, m0, n0, R;
  __device__ void operator()(int i, int j, double v) const {
    int x = m0 + i, r = n0 + j;
    if (x >= N || r >= R) return;
    int col = r / N, y = r - col * N;
    Y[(long)col * ldy + iperm[y * N + x]] = v;
  }
};

// Xh(p, r) = sum_x S(p,x) X[col*ldx + iperm[y*N + x]],  r = col*N + y
__global__ void __launch_bounds__(256) k_dst_fwd(const double* S, const double* X, int ldx, const int* iperm,
                                                 double* Xh, int N, int ncol) {
  __shared__ double smem[GCfg::LDS_DOUBLES];
  const int m0 = blockIdx.x * GBM, n0 = blockIdx.y * GBN;
  const int R = ncol * N;
  DstLS la{S, N, m0};
  DstLGather lb{X, ldx, iperm, N, n0, R};
  double acc[GTM][GTN];
  tile_zero<GBM, GBN, GTM, GTN>(acc);
  tile_gemm_acc<GBM, GBN, GBK, GTM, GTN>(la, lb, 0, N, acc, smem);
  DstStMode st{Xh, N, m0, n0, R};
  tile_store<GBM, GBN, GBK, GTM, GTN>(st, acc);
}

// Y[col*ldy + iperm[y*N + x]] = sum_p S(x,p) W(p, r)
__global__ void __launch_bounds__(256) k_dst_inv(const double* S, const double* W, const int* iperm, double* Y,
                                                 int ldy, int N, int ncol) {
  __shared__ double smem[GCfg::LDS_DOUBLES];
  const int m0 = blockIdx.x * GBM, n0 = blockIdx.y * GBN;
  const int R = ncol * N;
  DstLS la{S, N, m0};
  DstLMode lb{W, N, n0, R};
  double acc[GTM][GTN];
  tile_zero<GBM, GBN, GTM, GTN>(acc);
  tile_gemm_acc<GBM, GBN, GBK, GTM, GTN>(la, lb, 0, N, acc, smem);
  DstStScatter st{Y, ldy, iperm, N, m0, n0, R};
  tile_store<GBM, GBN, GBK, GTM, GTN>(st, acc);
}

// 1D gather / scatter between tree order (ld) and line order (ld n)
__global__ void k_gather(const double* X, int ldx, const int* iperm, double* Xg, int n, int ncol) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * ncol) return;
  int col = e / n, g = e % n;
  Xg[e] = X[(long)col * ldx + iperm[g]];
}
__global__ void k_scatter(const double* Wg, const int* iperm, double* Y, int ldy, int n, int ncol) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * ncol) return;
  int col = e / n, g = e % n;
  Y[(long)col * ldy + iperm[g]] = Wg[e];
}

static hm_status ensure_thomas(Model* m, double kappa, double alpha) {
  if (m->thomas_key[0] == kappa && m->thomas_key[1] == alpha) return HM_OK;
  const double h2inv = 1.0 / (m->h * m->h);
  hipLaunchKernelGGL(k_thomas_coef, dim3(ceil_div(m->Np, 64)), dim3(64), 0, m->stream, m->d_thomas, m->d_mu,
                     m->L, m->Np, kappa, alpha, h2inv);
  HM_LAUNCH_CHECK();
  m->thomas_key[0] = kappa;
  m->thomas_key[1] = alpha;
  return HM_OK;
}

hm_status kapply(Model* m, const double theta[4], const double* X, int ldx, int c, double* outK,
                 double* outKap, double* outAlp, int ldo) {
  if (c <= 0) return HM_OK;
  const double kappa = theta[0], alpha = theta[1], tau2 = theta[2], sigma2 = theta[3];
  HM_CHECK(ensure_thomas(m, kappa, alpha));
  const int n = m->n, N = m->N;
  double* Xh = m->d_ws;
  double* W = m->d_ws + (long)n * m->cmax;
  double* Tk = m->d_ws + 2L * n * m->cmax;
  double* Ta = m->d_ws + 3L * n * m->cmax;
  const int mode = (outK ? 1 : 0) | (outKap ? 2 : 0) | (outAlp ? 4 : 0);
  const double h2inv = 1.0 / (m->h * m->h);
  for (int c0 = 0; c0 < c; c0 += m->cmax) {
    const int cc = std::min(m->cmax, c - c0);
    const double* Xc = X + (long)c0 * ldx;
    if (m->dim == 2) {
      dim3 g(ceil_div(N, GBM), ceil_div((long)cc * N, GBN));
      hipLaunchKernelGGL(k_dst_fwd, g, dim3(GCfg::NT), 0, m->stream, m->d_dst, Xc, ldx, m->d_iperm, Xh, N, cc);
    } else {
      hipLaunchKernelGGL(k_gather, dim3(ceil_div((long)n * cc, 256)), dim3(256), 0, m->stream, Xc, ldx,
                         m->d_iperm, Xh, n, cc);
    }
    HM_LAUNCH_CHECK();
    const int nthreads = cc * m->Np;
    dim3 tg(ceil_div(nthreads, 64)), tb(64);
#define HM_CHAIN(MD)                                                                                   \
  hipLaunchKernelGGL((k_thomas_chain<MD>), tg, tb, 0, m->stream, Xh, W, Tk, Ta, cc, n, m->L, m->Np,       \
                     m->d_thomas, m->d_mu, kappa, alpha, sigma2, tau2, h2inv)
    // the value chain always runs (tangents reuse its intermediates)
    switch (mode | 1) {
      case 1: HM_CHAIN(1); break;
      case 3: HM_CHAIN(3); break;
      case 5: HM_CHAIN(5); break;
      case 7: HM_CHAIN(7); break;
      default: break;
    }
#undef HM_CHAIN
    HM_LAUNCH_CHECK();
    double* outs[3] = {outK, outKap, outAlp};
    double* bufs[3] = {W, Tk, Ta};
    for (int q = 0; q < 3; ++q) {
      if (!outs[q]) continue;
      double* Yc = outs[q] + (long)c0 * ldo;
      if (m->dim == 2) {
        dim3 g(ceil_div(N, GBM), ceil_div((long)cc * N, GBN));
        hipLaunchKernelGGL(k_dst_inv, g, dim3(GCfg::NT), 0, m->stream, m->d_dst, bufs[q], m->d_iperm, Yc, ldo,
                           N, cc);
      } else {
        hipLaunchKernelGGL(k_scatter, dim3(ceil_div((long)n * cc, 256)), dim3(256), 0, m->stream, bufs[q],
                           m->d_iperm, Yc, ldo, n, cc);
      }
      HM_LAUNCH_CHECK();
    }
  }
  return HM_OK;
}

hm_status model_tables(Model* m) {
  const int n = m->n, N = m->N;
  hipLaunchKernelGGL(k_perm, dim3(ceil_div(n, 256)), dim3(256), 0, m->stream, m->d_perm, m->d_iperm, n, N,
                     m->dim, m->levels, m->nl);
  HM_LAUNCH_CHECK();
  int cnt = (m->dim == 2) ? N * N : N;
  hipLaunchKernelGGL(k_tables, dim3(ceil_div(cnt, 256)), dim3(256), 0, m->stream, m->d_dst, m->d_mu, N, m->dim);
  HM_LAUNCH_CHECK();
  return HM_OK;
}

}  // namespace hm
