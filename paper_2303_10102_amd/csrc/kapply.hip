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
#include "hm_trace.h"

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

__global__ void k_tables(double* S, double* mu, int N, int dim, double h) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  const double scale = sqrt(2.0 / (N + 1));
  if (e < N * N) {
    int p = e % N, x = e / N;
    long m = (long)(p + 1) * (x + 1) % (2L * (N + 1));
    S[e] = scale * sinpi((double)m / (double)(N + 1));
  }
  if (e < N) {
    double s = sinpi((double)(e + 1) / (2.0 * (N + 1)));
    mu[e] = 4.0 / (h * h) * s * s;
  }
}

// Even/odd halves of S for even N (H = N / 2).  The DST-I matrix obeys
// S(p, N-1-x) = (-1)^p S(p, x): on an axis that is transformed whole, the forward
// transform folds the input (a point plus its mirror for even modes, minus it for
// odd modes) and sums over H points only; the inverse forms the even-mode and
// odd-mode sums at the first H points and unfolds them (sum at x, difference at
// N-1-x).  Both halve the transform's multiply-adds.
//   P_par[i + k H] = S(2i + par, k),   Q_par[x + k H] = S(x, 2k + par),   i, k, x < H
// stored as P0, P1, Q0, Q1 at offsets 0, H^2, 2 H^2, 3 H^2.
__global__ void k_tables_half(double* Ph, int N) {
  const int H = N / 2;
  const long HH = (long)H * H;
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 4 * HH) return;
  const int t = (int)(e / HH);
  const long f = e % HH;
  const int a = (int)(f % H), b = (int)(f / H), par = t & 1;
  // P: row mode 2a + par, point b;  Q: point a, mode 2b + par
  const int mode = (t < 2) ? 2 * a + par : 2 * b + par;
  const int x = (t < 2) ? b : a;
  const long m = (long)(mode + 1) * (x + 1) % (2L * (N + 1));
  Ph[e] = sqrt(2.0 / (N + 1)) * sinpi((double)m / (double)(N + 1));
}

// Per-mode multipliers of the physics part of K (sigma2 A^-1 B^-2 A^-1; the nugget is
// added row by row, see kapply_multi), dK/dkappa, dK/dalpha: lam[o*N*Ny + p + q*N]
__global__ void k_mode_scale(double* lam, const double* mu, int N, int Ny, double kappa, double alpha,
                             double tau2, double sigma2) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * Ny) return;
  int p = e % N, q = e / N;
  double m = mu[p] + (Ny > 1 ? mu[q] : 0.0);
  double a = 1.0 + alpha * m, b = kappa * kappa + m;
  double l = sigma2 / (a * a * b * b);
  const long NN = (long)N * Ny;
  lam[e] = l;   // physics only: the nugget tau2 X is added outside the transforms
  lam[NN + e] = -4.0 * kappa * l / b;
  lam[2 * NN + e] = -2.0 * m * l / a;
}

// ---------------------------------------------------------------------------
// sine transforms with the tree<->grid reordering computed in the loads
//
// Axis maps.  A sketch pass at depth l reads an input that is zero outside one
// side (left or right children) of the depth-l split and needs the output only on
// the other side; both sides are alternating chunks of width W along the split
// axis.  AxisMap{W, par} enumerates the coordinates t -> (t / W) 2W + par W + t % W
// (the chunks of parity par); W = 0 is the whole axis.  The transforms then run
// over the compact half: the forward x-transform sums only the input's x, the
// y-transforms only the input's / needed y, the inverse x-transform writes only
// the needed x.  The quotient uses a reciprocal multiplier: for t < 2^16 and
// W <= 2^16, t / W = umulhi(t, ceil(2^32 / W)) exactly.
// ---------------------------------------------------------------------------
struct AxisMap {
  int W, par;
  unsigned mw;
  __host__ __device__ int operator()(int t) const {
#ifdef __HIP_DEVICE_COMPILE__
    if (!W) return t;
    const int q = (int)__umulhi((unsigned)t, mw);
    return q * 2 * W + par * W + (t - q * W);
#else
    return W ? (t / W) * 2 * W + par * W + t % W : t;
#endif
  }
  __host__ __device__ int extent(int n) const { return W ? n / 2 : n; }
};
static inline unsigned recip32(int w) { return w > 0 ? (unsigned)((0x100000000ULL + (unsigned)w - 1) / (unsigned)w) : 0u; }
static inline AxisMap axis_map(int W, int par) { return AxisMap{W, par, recip32(W)}; }

// The outputs of one K-apply (K X, dK/dkappa X, dK/dalpha X, any subset) share the
// forward transforms; their inverse transforms run as one launch, output o taking the
// multipliers lam[o] and writing Y[o] (x inverse) or slot o of the scratch (y inverse).
// Output o covers the first cols[o] columns of the block (a tangent may be wanted for
// fewer columns than the value); z-slices and column tiles of the launches are laid out
// output after output (zoff, toff: prefix sums of the columns and of the column tiles).
struct MultiOut {
  double* Y[3];
  const double* lam[3];
  long in_stride;    // input offset between outputs (0: one shared input)
  int nq;
  int cols[3], zoff[3], toff[3];
  __device__ __forceinline__ const double* lam_of(int o) const { return o == 0 ? lam[0] : (o == 1 ? lam[1] : lam[2]); }
  __device__ __forceinline__ double* y_of(int o) const { return o == 0 ? Y[0] : (o == 1 ? Y[1] : Y[2]); }
  __device__ __forceinline__ int pick(int v, const int (&off)[3]) const {
    return (nq > 2 && v >= off[2]) ? 2 : ((nq > 1 && v >= off[1]) ? 1 : 0);
  }
  __device__ __forceinline__ int get(const int (&a)[3], int o) const { return o == 0 ? a[0] : (o == 1 ? a[1] : a[2]); }
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
// Column geometry shared by the loaders and stores that address tree-ordered data:
// columns r = n0 + j < R of the compact (col, y') enumeration; an index past R maps
// to (0, 0) so that its dummy load stays inside the operand.
template <int AM>
struct ColGeo {
  int Ny, n0, R, colt, yt;
  __device__ __forceinline__ bool at(int j, int& col, int& y) const {
    const int r = n0 + j;
    if (r >= R) { col = 0; y = 0; return false; }
    split_col<AM>(r, Ny, colt, yt, j, col, y);
    return true;
  }
};
template <int AM>
__device__ __forceinline__ ColGeo<AM> col_geo(int Ny, int n0, int ncol) {
  const int colt = (AM == 1) ? n0 / Ny : 0, yt = (AM == 1) ? n0 - colt * Ny : 0;
  return ColGeo<AM>{Ny, n0, ncol * Ny, colt, yt};
}

struct DstLS {  // A(i, k) = S(m0 + i, xmap(k))   (S symmetric, N x N)
  const double* S; int N, m0; AxisMap xm;
  static constexpr bool kfast = false;
  static constexpr int NR = 1;
  __device__ bool load(int i, int k, double (&r)[1]) const {
    const int p = m0 + i;
    const bool ok = p < N;
    r[0] = S[(ok ? p : 0) + (long)xm(k) * N];
    return ok;
  }
  __device__ double fin(const double (&r)[1]) const { return r[0]; }
};
struct DstLSrow {  // A(i, k) = S(xmap(m0 + i), k) for m0 + i < Mx
  const double* S; int N, m0, Mx; AxisMap xm;
  static constexpr bool kfast = false;
  static constexpr int NR = 1;
  __device__ bool load(int i, int k, double (&r)[1]) const {
    const int x = m0 + i;
    const bool ok = x < Mx;
    r[0] = S[xm(ok ? x : 0) + (long)k * N];
    return ok;
  }
  __device__ double fin(const double (&r)[1]) const { return r[0]; }
};
template <int AM>
struct DstLGather {  // B(k, j) = X[col ldx + tree(xmap(k), ymap(y'))]
  const double* X; int ldx; TreeIdx tix; ColGeo<AM> cg; AxisMap xm, ym;
  static constexpr bool kfast = true;
  static constexpr int NR = 1;
  __device__ bool load(int k, int j, double (&r)[1]) const {
    int col, y;
    const bool ok = cg.at(j, col, y);
    r[0] = X[(long)col * ldx + tix(xm(k), ym(y))];
    return ok;
  }
  __device__ double fin(const double (&r)[1]) const { return r[0]; }
};
template <int AM, bool LAM>
struct DstLMode {  // B(p, r) = W[p + r N], times lam[p + ymap(y') N] when LAM (1D: lam[p])
  const double* W; const double* lam; int N; ColGeo<AM> cg; AxisMap ym;
  static constexpr bool kfast = true;
  static constexpr int NR = LAM ? 2 : 1;
  __device__ bool load(int k, int j, double (&r)[NR]) const {
    int col, y;
    const bool ok = cg.at(j, col, y);
    const int rr = ok ? cg.n0 + j : 0;
    r[0] = W[k + (long)rr * N];
    if constexpr (LAM) r[1] = lam[k + (long)ym(y) * N];
    return ok;
  }
  __device__ double fin(const double (&r)[NR]) const {
    if constexpr (LAM) return r[0] * r[1];
    else return r[0];
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
struct DstStScatter {  // Y[col ldy + tree(xmap(x'), ymap(y'))]
  double* Y; int ldy; TreeIdx tix; ColGeo<AM> cg; int m0, Mx; AxisMap xm, ym;
  __device__ void operator()(int i, int j, double v) const {
    const int xi = m0 + i;
    int col, y;
    if (xi >= Mx || !cg.at(j, col, y)) return;
    Y[(long)col * ldy + tix(xm(xi), ym(y))] = v;
  }
};
// y-direction transforms of every column's N x Nyin block M (rows p, cols y'):
//   forward  C_c(p, q)  = sum_{y'} M_c(p, y') S(ymap(y'), q)          (Nyin compact, q full)
//   inverse  C_c(p, y') = sum_q (lam o M_c)(p, q) S(q, ymap(y'))      (q full, y' compact)
template <bool LAM>
struct DyLA {
  const double* M; const double* lam; int N, m0;
  static constexpr bool kfast = false;
  static constexpr int NR = LAM ? 2 : 1;
  __device__ bool load(int i, int k, double (&r)[NR]) const {
    const int p = m0 + i;
    const bool ok = p < N;
    const long e = (ok ? p : 0) + (long)k * N;
    r[0] = M[e];
    if constexpr (LAM) r[1] = lam[e];
    return ok;
  }
  __device__ double fin(const double (&r)[NR]) const {
    if constexpr (LAM) return r[0] * r[1];
    else return r[0];
  }
};
struct DyLBfwd {  // B(k, j) = S(ymap(k), n0 + j)
  const double* S; int N, n0; AxisMap ym;
  static constexpr bool kfast = true;
  static constexpr int NR = 1;
  __device__ bool load(int k, int j, double (&r)[1]) const {
    const int q = n0 + j;
    const bool ok = q < N;
    r[0] = S[ym(k) + (long)(ok ? q : 0) * N];
    return ok;
  }
  __device__ double fin(const double (&r)[1]) const { return r[0]; }
};
struct DyLBinv {  // B(k, j) = S(k, ymap(n0 + j)) for n0 + j < Nout
  const double* S; int N, n0, Nout; AxisMap ym;
  static constexpr bool kfast = true;
  static constexpr int NR = 1;
  __device__ bool load(int k, int j, double (&r)[1]) const {
    const int c = n0 + j;
    const bool ok = c < Nout;
    r[0] = S[k + (long)ym(ok ? c : 0) * N];
    return ok;
  }
  __device__ double fin(const double (&r)[1]) const { return r[0]; }
};

// Xh(p, r) = sum_{x'} S(p, xmap(x')) X[col ldx + tree(xmap(x'), ymap(y'))],  r = col Ny + y'
template <int AM>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k_dst_fwd(const double* S, const double* X, int ldx, TreeIdx tix,
          double* Xh, int N, int Ny, int ncol, int Kx, AxisMap xm,
          AxisMap ym) {
  __shared__ double smem[GSMEM];
  const TileIdx tb = tile_block();
  const int m0 = tb.x * GBM, n0 = tb.y * GBN;
  const ColGeo<AM> cg = col_geo<AM>(Ny, n0, ncol);
  DstLS la{S, N, m0, xm};
  DstLGather<AM> lb{X, ldx, tix, cg, xm, ym};
  TileAcc acc;
  tile_zero(acc);
  tile_gemm(la, lb, 0, Kx, acc, smem);
  tile_store(DstStMode{Xh, N, m0, n0, cg.R}, acc);
}

// forward y: C_c = M_c S[ymap(.), :]  (M_c: N x Nyin at c*N*Nyin; C_c: N x N at c*N*N)
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k_dst_yf(const double* S, const double* M, double* C, int N, int Nyin,
         AxisMap ym) {
  __shared__ double smem[GSMEM];
  const TileIdx tb = tile_block();
  const int m0 = tb.x * GBM, n0 = tb.y * GBN;
  DyLA<false> la{M + (long)tb.z * N * Nyin, nullptr, N, m0};
  DyLBfwd lb{S, N, n0, ym};
  TileAcc acc;
  tile_zero(acc);
  tile_gemm(la, lb, 0, Nyin, acc, smem);
  DstStMode st{C + (long)tb.z * N * N, N, m0, n0, N};
  tile_store(st, acc);
}

// inverse y: C_{o,c} = (lam_o o M_c) S[:, ymap(.)]  (M_c: N x N; C_{o,c}: N x Nyout at
// o * cslot + c*N*Nyout); grid.z = outputs x columns
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k_dst_yi(const double* S, const double* M, MultiOut mo, double* C,
         long cslot, int N, int Nyout, AxisMap ym) {
  __shared__ double smem[GSMEM];
  const TileIdx tb = tile_block();
  const int m0 = tb.x * GBM, n0 = tb.y * GBN;
  const int o = mo.pick(tb.z, mo.zoff), c = tb.z - mo.get(mo.zoff, o);
  DyLA<true> la{M + (long)c * N * N, mo.lam_of(o), N, m0};
  DyLBinv lb{S, N, n0, Nyout, ym};
  TileAcc acc;
  tile_zero(acc);
  tile_gemm(la, lb, 0, N, acc, smem);
  DstStMode st{C + o * cslot + (long)c * N * Nyout, N, m0, n0, Nyout};
  tile_store(st, acc);
}

// Y[col ldy + tree(xmap(x'), ymap(y'))] = sum_p S(xmap(x'), p) (lam o W)(p, r)
// grid.y = outputs x column tiles
template <int AM, bool LAM>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k_dst_inv(const double* S, const double* W, MultiOut mo, TreeIdx tix,
          int ldy, int N, int Ny, int Mx, AxisMap xm, AxisMap ym) {
  __shared__ double smem[GSMEM];
  const TileIdx tb = tile_block();
  const int o = mo.pick(tb.y, mo.toff);
  const int ncol = mo.get(mo.cols, o);
  const int m0 = tb.x * GBM, n0 = (tb.y - mo.get(mo.toff, o)) * GBN;
  const ColGeo<AM> cg = col_geo<AM>(Ny, n0, ncol);
  double* Y = mo.y_of(o);
  DstLSrow la{S, N, m0, Mx, xm};
  DstLMode<AM, LAM> lb{W + o * mo.in_stride, mo.lam_of(o), N, cg, ym};
  TileAcc acc;
  tile_zero(acc);
  tile_gemm(la, lb, 0, N, acc, smem);
  tile_store(DstStScatter<AM>{Y, ldy, tix, cg, m0, Mx, xm, ym}, acc);
}

// ---- folded transforms (even N, the transformed axis whole) ------------------
struct HalfA {  // A(i, k) = Tab[m0 + i + k H] for m0 + i < H   (P_par or Q_par)
  const double* T; int H, m0;
  static constexpr bool kfast = false;
  static constexpr int NR = 1;
  __device__ bool load(int i, int k, double (&r)[1]) const {
    const int row = m0 + i;
    const bool ok = row < H;
    r[0] = T[(ok ? row : 0) + (long)k * H];
    return ok;
  }
  __device__ double fin(const double (&r)[1]) const { return r[0]; }
};
struct HalfB {  // B(k, j) = Tab[k + (n0 + j) H] for n0 + j < H
  const double* T; int H, n0;
  static constexpr bool kfast = true;
  static constexpr int NR = 1;
  __device__ bool load(int k, int j, double (&r)[1]) const {
    const int c = n0 + j;
    const bool ok = c < H;
    r[0] = T[k + (long)(ok ? c : 0) * H];
    return ok;
  }
  __device__ double fin(const double (&r)[1]) const { return r[0]; }
};
template <int AM>
struct DstLGatherFold {  // B(k, j) = X(x = k) + sgn X(x = N-1-k) of column r = n0 + j
  const double* X; int ldx; TreeIdx tix; ColGeo<AM> cg; int N; AxisMap ym; double sgn;
  static constexpr bool kfast = true;
  static constexpr int NR = 2;
  __device__ bool load(int k, int j, double (&r)[2]) const {
    int col, y;
    const bool ok = cg.at(j, col, y);
    const double* Xc = X + (long)col * ldx;
    const int yy = ym(y);
    r[0] = Xc[tix(k, yy)];
    r[1] = Xc[tix(N - 1 - k, yy)];
    return ok;
  }
  __device__ double fin(const double (&r)[2]) const { return r[0] + sgn * r[1]; }
};
struct DyLAFold {  // A(i, k) = M(p, k) + sgn M(p, N-1-k), p = m0 + i
  const double* M; int N, m0; double sgn;
  static constexpr bool kfast = false;
  static constexpr int NR = 2;
  __device__ bool load(int i, int k, double (&r)[2]) const {
    const int p = m0 + i;
    const bool ok = p < N;
    const int pp = ok ? p : 0;
    r[0] = M[pp + (long)k * N];
    r[1] = M[pp + (long)(N - 1 - k) * N];
    return ok;
  }
  __device__ double fin(const double (&r)[2]) const { return r[0] + sgn * r[1]; }
};
struct DyLApar {  // A(i, k) = (lam o M)(p, 2k + par), p = m0 + i
  const double* M; const double* lam; int N, m0, par;
  static constexpr bool kfast = false;
  static constexpr int NR = 2;
  __device__ bool load(int i, int k, double (&r)[2]) const {
    const int p = m0 + i;
    const bool ok = p < N;
    const long e = (ok ? p : 0) + (long)(2 * k + par) * N;
    r[0] = M[e];
    r[1] = lam[e];
    return ok;
  }
  __device__ double fin(const double (&r)[2]) const { return r[0] * r[1]; }
};
template <int AM, bool LAM>
struct DstLModePar {  // B(k, j) = W(2k + par, r) (times lam(2k + par, ymap(y')) when LAM), r = n0 + j
  const double* W; const double* lam; int N, par; ColGeo<AM> cg; AxisMap ym;
  static constexpr bool kfast = true;
  static constexpr int NR = LAM ? 2 : 1;
  __device__ bool load(int k, int j, double (&r)[NR]) const {
    int col, y;
    const bool ok = cg.at(j, col, y);
    const int rr = ok ? cg.n0 + j : 0;
    const int p = 2 * k + par;
    r[0] = W[p + (long)rr * N];
    if constexpr (LAM) r[1] = lam[p + (long)ym(y) * N];
    return ok;
  }
  __device__ double fin(const double (&r)[NR]) const {
    if constexpr (LAM) return r[0] * r[1];
    else return r[0];
  }
};
struct DstStModePar {  // Xh(2(m0 + i) + par, r)
  double* p; int N, H, m0, n0, R, par;
  __device__ void operator()(int i, int j, double v) const {
    const int ii = m0 + i, r = n0 + j;
    if (ii < H && r < R) p[2 * ii + par + (long)r * N] = v;
  }
};
struct DyStColPar {  // C(p, 2(n0 + j) + par)
  double* C; int N, H, m0, n0, par;
  __device__ void operator()(int i, int j, double v) const {
    const int pp = m0 + i, jj = n0 + j;
    if (pp < N && jj < H) C[pp + (long)(2 * jj + par) * N] = v;
  }
};
struct DyStUnfold {  // C(p, y') = e + o, C(p, N-1-y') = e - o, y' = n0 + j < H
  double* C; int N, H, m0, n0;
  __device__ void operator()(int i, int j, double e, double o) const {
    const int pp = m0 + i, y = n0 + j;
    if (pp < N && y < H) {
      C[pp + (long)y * N] = e + o;
      C[pp + (long)(N - 1 - y) * N] = e - o;
    }
  }
};
template <int AM>
struct DstStScatterUnfold {  // Y at (x, r) = e + o and (N-1-x, r) = e - o, x = m0 + i < H
  double* Y; int ldy; TreeIdx tix; ColGeo<AM> cg; int N, H, m0; AxisMap ym;
  __device__ void operator()(int i, int j, double e, double o) const {
    const int x = m0 + i;
    int col, y;
    if (x >= H || !cg.at(j, col, y)) return;
    double* Yc = Y + (long)col * ldy;
    const int yy = ym(y);
    Yc[tix(x, yy)] = e + o;
    Yc[tix(N - 1 - x, yy)] = e - o;
  }
};

// forward x, x whole: Xh(2i + par, r) = sum_{x < H} P_par(i, x) (X(x) +- X(N-1-x))
// grid.x: 2 * ht tiles (parity major), grid.y: column tiles
template <int AM>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k_dst_fwd_fold(const double* Ph, const double* X, int ldx, TreeIdx tix,
               double* Xh, int N, int Ny, int ncol, AxisMap ym) {
  __shared__ double smem[GSMEM];
  const TileIdx tb = tile_block();
  const int H = N / 2, ht = (H + GBM - 1) / GBM;
  const int par = tb.x >= ht ? 1 : 0;
  const int m0 = (tb.x - par * ht) * GBM, n0 = tb.y * GBN;
  const ColGeo<AM> cg = col_geo<AM>(Ny, n0, ncol);
  HalfA la{Ph + (long)par * H * H, H, m0};
  DstLGatherFold<AM> lb{X, ldx, tix, cg, N, ym, par ? -1.0 : 1.0};
  TileAcc acc;
  tile_zero(acc);
  tile_gemm(la, lb, 0, H, acc, smem);
  tile_store(DstStModePar{Xh, N, H, m0, n0, cg.R, par}, acc);
}

// forward y, y whole: C_c(p, 2j + par) = sum_{y < H} (M_c(p, y) +- M_c(p, N-1-y)) Q_par(y, j)
// grid.y: 2 * ht tiles (parity major)
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k_dst_yf_fold(const double* Ph, const double* M, double* C, int N) {
  __shared__ double smem[GSMEM];
  const TileIdx tb = tile_block();
  const int H = N / 2, ht = (H + GBN - 1) / GBN;
  const int par = tb.y >= ht ? 1 : 0;
  const int m0 = tb.x * GBM, n0 = (tb.y - par * ht) * GBN;
  const long NN = (long)N * N;
  DyLAFold la{M + tb.z * NN, N, m0, par ? -1.0 : 1.0};
  HalfB lb{Ph + (long)(2 + par) * H * H, H, n0};
  TileAcc acc;
  tile_zero(acc);
  tile_gemm(la, lb, 0, H, acc, smem);
  tile_store(DyStColPar{C + tb.z * NN, N, H, m0, n0, par}, acc);
}

// inverse y, y whole: e = sum_k (lam o M_c)(p, 2k) P0(k, y'), o = the odd modes with P1;
// C_c(p, y') = e + o, C_c(p, N-1-y') = e - o for y' < H
// (grid.z = outputs x columns, as k_dst_yi)
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
k_dst_yi_fold(const double* Ph, const double* M, MultiOut mo, double* C,
              long cslot, int N) {
  __shared__ double smem[GSMEM];
  const TileIdx tb = tile_block();
  const int H = N / 2;
  const int m0 = tb.x * GBM, n0 = tb.y * GBN;
  const int q = mo.pick(tb.z, mo.zoff), c = tb.z - mo.get(mo.zoff, q);
  const long NN = (long)N * N, HH = (long)H * H;
  const double* Mz = M + c * NN;
  const double* lam = mo.lam_of(q);
  TileAcc e, o;
  tile_zero(e);
  tile_zero(o);
  tile_gemm(DyLApar{Mz, lam, N, m0, 0}, HalfB{Ph, H, n0}, 0, H, e, smem);
  tile_gemm(DyLApar{Mz, lam, N, m0, 1}, HalfB{Ph + HH, H, n0}, 0, H, o, smem);
  tile_store2(DyStUnfold{C + q * cslot + c * NN, N, H, m0, n0}, e, o);
}

// inverse x, x whole: e = sum_k Q0(x, k) W(2k, r), o = sum_k Q1(x, k) W(2k+1, r) (W scaled
// by lam when LAM, the 1D case); Y(x) = e + o, Y(N-1-x) = e - o for x < H
// (grid.y = outputs x column tiles, as k_dst_inv)
template <int AM, bool LAM>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
k_dst_inv_fold(const double* Ph, const double* W, MultiOut mo, TreeIdx tix,
               int ldy, int N, int Ny, AxisMap ym) {
  __shared__ double smem[GSMEM];
  const TileIdx tb = tile_block();
  const int H = N / 2;
  const long HH = (long)H * H;
  const int q = mo.pick(tb.y, mo.toff);
  const int ncol = mo.get(mo.cols, q);
  const int m0 = tb.x * GBM, n0 = (tb.y - mo.get(mo.toff, q)) * GBN;
  const ColGeo<AM> cg = col_geo<AM>(Ny, n0, ncol);
  const double* Wq = W + q * mo.in_stride;
  const double* lam = mo.lam_of(q);
  TileAcc e, o;
  tile_zero(e);
  tile_zero(o);
  tile_gemm(HalfA{Ph + 2 * HH, H, m0}, DstLModePar<AM, LAM>{Wq, lam, N, 0, cg, ym}, 0, H, e, smem);
  tile_gemm(HalfA{Ph + 3 * HH, H, m0}, DstLModePar<AM, LAM>{Wq, lam, N, 1, cg, ym}, 0, H, o, smem);
  tile_store2(DstStScatterUnfold<AM>{mo.y_of(q), ldy, tix, cg, N, H, m0, ym}, e, o);
}

hm_status ensure_scale(Model* m, const double* theta) {
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
  xm = axis_map(0, 0);
  ym = axis_map(0, 0);
  // the sides of a non-uniform bisection are not alternating chunks of one width:
  // whole transforms there (the output is then written on every row)
  if (sel.mode == 0 || !m->uniform) return;
  int w = m->N, h = (m->dim == 2) ? m->N : 1;
  bool xsplit = true;
  for (int d = 1; d <= sel.depth; ++d) {
    if (w >= h) { w /= 2; xsplit = true; }
    else { h /= 2; xsplit = false; }
  }
  const AxisMap am = axis_map(xsplit ? w : h, sel.mode == 2 ? 1 : 0);
  if (xsplit) xm = am;
  else ym = am;
}

// Transform launches for one block of cc columns.  An axis transformed whole (map
// W = 0) of even length runs folded (half the multiply-adds); a compact half, or
// an odd N, runs the plain GEMM over the points it has.
static int amode(int ny) { return ny == 1 ? 2 : (ny % GBN == 0 ? 1 : 0); }
static inline bool folds(const Model* m, AxisMap am) { return m->d_dsth && am.W == 0; }
#define HM_DST_LAUNCH(kern, g, ...) hipLaunchKernelGGL(kern, g, dim3(GCfg::NT), 0, m->stream, __VA_ARGS__)

// Xh (N x cc*Ny) = S_x applied to the gathered columns (x compact per xm, y per ym)
static void x_forward(Model* m, const double* X, int ldx, double* Xh, int cc, int Ny, AxisMap xm, AxisMap ym) {
  const int N = m->N, am = amode(Ny);
  if (folds(m, xm)) {
    const int H = N / 2;
    dim3 g(2 * ceil_div(H, GBM), ceil_div((long)cc * Ny, GBN));
    if (am == 2) HM_DST_LAUNCH((k_dst_fwd_fold<2>), g, m->d_dsth, X, ldx, m->tix, Xh, N, Ny, cc, ym);
    else if (am == 1) HM_DST_LAUNCH((k_dst_fwd_fold<1>), g, m->d_dsth, X, ldx, m->tix, Xh, N, Ny, cc, ym);
    else HM_DST_LAUNCH((k_dst_fwd_fold<0>), g, m->d_dsth, X, ldx, m->tix, Xh, N, Ny, cc, ym);
    return;
  }
  const int Kx = xm.extent(N);
  dim3 g(ceil_div(N, GBM), ceil_div((long)cc * Ny, GBN));
  if (am == 2) HM_DST_LAUNCH((k_dst_fwd<2>), g, m->d_dst, X, ldx, m->tix, Xh, N, Ny, cc, Kx, xm, ym);
  else if (am == 1) HM_DST_LAUNCH((k_dst_fwd<1>), g, m->d_dst, X, ldx, m->tix, Xh, N, Ny, cc, Kx, xm, ym);
  else HM_DST_LAUNCH((k_dst_fwd<0>), g, m->d_dst, X, ldx, m->tix, Xh, N, Ny, cc, Kx, xm, ym);
}
// C_c (N x N) = M_c (N x Nyin, compact per ym) transformed along y, for cc columns
static void y_forward(Model* m, const double* M, double* C, int cc, AxisMap ym) {
  const int N = m->N;
  if (folds(m, ym)) {
    dim3 g(ceil_div(N, GBM), 2 * ceil_div(N / 2, GBN), cc);
    HM_DST_LAUNCH(k_dst_yf_fold, g, m->d_dsth, M, C, N);
    return;
  }
  dim3 g(ceil_div(N, GBM), ceil_div(N, GBN), cc);
  HM_DST_LAUNCH(k_dst_yf, g, m->d_dst, M, C, N, ym.extent(N), ym);
}
// C_{o,c} (N x Nyout, compact per ym; output o at C + o * cslot) = (lam_o o M_c)
// transformed back along y, c < cols[o], all outputs in one launch
static void y_inverse(Model* m, const double* M, MultiOut mo, double* C, long cslot, AxisMap ym) {
  const int N = m->N;
  int z = 0;
  for (int o = 0; o < mo.nq; ++o) {
    mo.zoff[o] = z;
    z += mo.cols[o];
  }
  if (folds(m, ym)) {
    dim3 g(ceil_div(N, GBM), ceil_div(N / 2, GBN), z);
    HM_DST_LAUNCH(k_dst_yi_fold, g, m->d_dsth, M, mo, C, cslot, N);
    return;
  }
  const int Nyo = ym.extent(N);
  dim3 g(ceil_div(N, GBM), ceil_div(Nyo, GBN), z);
  HM_DST_LAUNCH(k_dst_yi, g, m->d_dst, M, mo, C, cslot, N, Nyo, ym);
}
// Y_o (scattered to tree order; x compact per xm) = S_x applied to the first cols[o]
// column groups of W + o * mo.in_stride (N x cols*Ny), scaled by lam_o when LAM
// (one-dimensional models); all outputs in one launch
static void x_inverse(Model* m, const double* W, MultiOut mo, bool lam, int ldy, int Ny, AxisMap xm, AxisMap ym) {
  const int N = m->N, am = amode(Ny);
  const TreeIdx tix = m->tix;
  int t = 0;
  for (int o = 0; o < mo.nq; ++o) {
    mo.toff[o] = t;
    t += ceil_div((long)mo.cols[o] * Ny, GBN);
  }
  if (folds(m, xm)) {
    dim3 g(ceil_div(N / 2, GBM), t);
    if (am == 2 && lam) HM_DST_LAUNCH((k_dst_inv_fold<2, true>), g, m->d_dsth, W, mo, tix, ldy, N, Ny, ym);
    else if (am == 2) HM_DST_LAUNCH((k_dst_inv_fold<2, false>), g, m->d_dsth, W, mo, tix, ldy, N, Ny, ym);
    else if (am == 1) HM_DST_LAUNCH((k_dst_inv_fold<1, false>), g, m->d_dsth, W, mo, tix, ldy, N, Ny, ym);
    else HM_DST_LAUNCH((k_dst_inv_fold<0, false>), g, m->d_dsth, W, mo, tix, ldy, N, Ny, ym);
    return;
  }
  const int Mx = xm.extent(N);
  dim3 g(ceil_div(Mx, GBM), t);
  if (am == 2 && lam) HM_DST_LAUNCH((k_dst_inv<2, true>), g, m->d_dst, W, mo, tix, ldy, N, Ny, Mx, xm, ym);
  else if (am == 2) HM_DST_LAUNCH((k_dst_inv<2, false>), g, m->d_dst, W, mo, tix, ldy, N, Ny, Mx, xm, ym);
  else if (am == 1) HM_DST_LAUNCH((k_dst_inv<1, false>), g, m->d_dst, W, mo, tix, ldy, N, Ny, Mx, xm, ym);
  else HM_DST_LAUNCH((k_dst_inv<0, false>), g, m->d_dst, W, mo, tix, ldy, N, Ny, Mx, xm, ym);
}
#undef HM_DST_LAUNCH

// Y[t, j] = 0 on the padding rows t (perm[t] < 0), j < c.
__global__ void k_zero_pad_rows(double* Y, int ldy, const int* perm, int n, int c) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * c) return;
  const int t = (int)(e % n), j = (int)(e / n);
  if (perm[t] < 0) Y[t + (long)j * ldy] = 0.0;
}

// Y[t, j] += tau2 X[t, j] for the rows t of the leaves selected by (mode, depth), j < c.
// Padding rows (perm[t] < 0; perm null for a uniform tree) are skipped; rows whose
// natural index is >= split (the second variable of the bivariate model) take tau2b.
__global__ void k_nugget(double* Y, int ldy, const double* X, int ldx, int n, int nl, int c, double tau2,
                         double tau2b, long split, int levels, int mode, int depth, const int* perm) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * c) return;
  const int t = (int)(e % n), j = (int)(e / n);
  const int g = perm ? perm[t] : 0;
  if (g < 0) return;
  if (mode != 0) {
    const int anc = (t / nl) >> (levels - depth);
    if (((anc & 1) == 0) != (mode == 1)) return;
  }
  Y[t + (long)j * ldy] += (g >= split ? tau2b : tau2) * X[t + (long)j * ldx];
}

// outK += tau2 X on the rows where the input and the wanted output overlap
static hm_status add_nugget(Model* m, const double* theta, const double* X, int ldx, double* outK, int cK, int ldo,
                            LeafSel in_sel, LeafSel out_sel) {
  const bool disjoint = in_sel.mode != 0 && out_sel.mode != 0 && in_sel.depth == out_sel.depth &&
                        in_sel.mode != out_sel.mode;
  if (!outK || cK <= 0 || disjoint) return HM_OK;
  const int n = m->n;
  const bool two = m->nvars == 2;
  hipLaunchKernelGGL(k_nugget, dim3(ceil_div((long)n * cK, 256)), dim3(256), 0, m->stream, outK, ldo, X, ldx, n, m->nl,
                     cK, theta[2], two ? theta[4] : theta[2], two ? m->nsplit : (long)m->n_real, m->levels,
                     out_sel.mode, out_sel.depth, m->uniform ? nullptr : m->d_perm);
  HM_LAUNCH_CHECK();
  return HM_OK;
}

// ---------------------------------------------------------------------------
// caller-supplied operator (hm_model_create_op): the columns are gathered into the
// caller's point order, the operator (and its derivatives) applied, and the results
// scattered back to tree order scaled by sigma2 (K = sigma2 K_op + tau2 I).
// ---------------------------------------------------------------------------
// Xn[i + j nr] = X[iperm[i] + j ldx]
__global__ void __launch_bounds__(256) k_gather_nat(const double* X, long ldx, double* Xn, const int* iperm, int nr, int c) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)nr * c) return;
  const int i = (int)(e % nr), j = (int)(e / nr);
  Xn[e] = X[iperm[i] + j * ldx];
}
// Y[t + j ldy] = s Yn[perm[t] + j nr] (0 on padding rows)
__global__ void k_scatter_tree(const double* Yn, double* Y, long ldy, const int* perm, int n, int nr, int c, double s) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * c) return;
  const int t = (int)(e % n), j = (int)(e / n), g = perm[t];
  Y[t + j * ldy] = g >= 0 ? s * Yn[g + (long)j * nr] : 0.0;
}

static hm_status op_call(Model* m, int which, const double* theta, const double* Xn, int c, double* Yn) {
  const int rc = m->op(m->op_ctx, which, theta, Xn, m->n_real, c, Yn, m->n_real, (void*)m->stream);
  if (rc != 0 && m->op_builtin) return (hm_status)rc;
  if (rc != 0) {
    set_error("the covariance operator callback failed (code " + std::to_string(rc) + ")");
    return HM_E_DEVICE;
  }
  HM_LAUNCH_CHECK();
  return HM_OK;
}

static hm_status op_kapply(Model* m, double* ws, int cblk, const double* theta, const double* X, int ldx, int c,
                           double* const outs[3], const int ocols[3], int ldo) {
  const int n = m->n, nr = m->n_real;
  cblk = std::min(cblk, m->cmax);   // operators see at most cmax columns at a time
  double* Xn = ws;
  double* Yn = ws + (long)n * cblk;
  for (int c0 = 0; c0 < c; c0 += cblk) {
    const int cc = std::min(cblk, c - c0);
    hipLaunchKernelGGL(k_gather_nat, dim3(ceil_div((long)nr * cc, 256)), dim3(256), 0, m->stream, X + (long)c0 * ldx,
                       (long)ldx, Xn, m->d_iperm, nr, cc);
    HM_LAUNCH_CHECK();
    for (int q = 0; q < 3; ++q) {
      const int oc = std::min(cc, ocols[q] - c0);
      if (!outs[q] || oc <= 0) continue;
      HM_CHECK(op_call(m, q, theta, Xn, oc, Yn));
      hipLaunchKernelGGL(k_scatter_tree, dim3(ceil_div((long)n * oc, 256)), dim3(256), 0, m->stream, Yn,
                         outs[q] + (long)c0 * ldo, (long)ldo, m->d_perm, n, nr, oc, theta[3]);
      HM_LAUNCH_CHECK();
    }
  }
  return HM_OK;
}

// The K-apply with its transform scratch ws (5 * n * cblk doubles) passed in, columns
// processed cblk at a time.
static hm_status kapply_core(Model* m, double* ws, int cblk, const double* theta, const double* X, int ldx, int c,
                             double* outK, int cK, double* outKap, int cKap, double* outAlp, int cAlp, int ldo,
                             LeafSel in_sel, LeafSel out_sel) {
  if (c <= 0) return HM_OK;
  m->cnt.kapply_calls += 1;
  m->cnt.kcols_value += outK ? cK : 0;
  m->cnt.kcols_deriv += (outKap ? cKap : 0) + (outAlp ? cAlp : 0);
  if (cK > c || cKap > c || cAlp > c) {
    set_error("kapply: an output wants more columns than the input has");
    return HM_E_INVAL;
  }
  if (m->op) {
    double* const outs_op[3] = {outK, outKap, outAlp};
    const int ocols_op[3] = {outK ? cK : 0, outKap ? cKap : 0, outAlp ? cAlp : 0};
    HM_CHECK(op_kapply(m, ws, cblk, theta, X, ldx, c, outs_op, ocols_op, ldo));
    return add_nugget(m, theta, X, ldx, outK, cK, ldo, in_sel, out_sel);
  }
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
  double* Xh = ws;                        // x-transformed (compact input y)
  double* X2 = ws + (long)n * cblk;       // x- and y-transformed (2D)
  double* X3 = ws + 2L * n * cblk;        // scaled and y-inverse-transformed, one slot per output
  double* outs[3] = {outK, outKap, outAlp};
  const int ocols[3] = {outK ? cK : 0, outKap ? cKap : 0, outAlp ? cAlp : 0};
  const bool pf = prof_on(m, PF_DST);
  double nout = 0.0;   // output columns per input column
  for (int q = 0; q < 3; ++q) nout += (double)ocols[q] / c;
  // work of the transform GEMMs actually run, per column (a folded axis halves its GEMM)
  const double fx_in = folds(m, xin) ? 0.5 : 1.0, fy_in = folds(m, yin) ? 0.5 : 1.0;
  const double fx_out = folds(m, xout) ? 0.5 : 1.0, fy_out = folds(m, yout) ? 0.5 : 1.0;
  const double fl_fwd = fx_in * 2.0 * N * Kx * Nyi + (two ? fy_in * 2.0 * N * Nyi * (double)N : 0.0);
  const double fl_out = (two ? fy_out * 2.0 * N * N * (double)Nyo : 0.0) + fx_out * 2.0 * Mx * N * (double)Nyo;
  const double per_col = fl_fwd + nout * fl_out;
  if (pf) prof_begin(m, PF_DST);
  for (int c0 = 0; c0 < c; c0 += cblk) {
    const int cc = std::min(cblk, c - c0);
    x_forward(m, X + (long)c0 * ldx, ldx, Xh, cc, Nyi, xin, yin);
    HM_LAUNCH_CHECK();
    if (two) {
      y_forward(m, Xh, X2, cc, yin);
      HM_LAUNCH_CHECK();
    }
    MultiOut mo{};
    for (int q = 0; q < 3; ++q) {
      const int oc = std::min(cc, ocols[q] - c0);   // this output's columns in the block
      if (!outs[q] || oc <= 0) continue;
      mo.Y[mo.nq] = outs[q] + (long)c0 * ldo;
      mo.lam[mo.nq] = m->d_lam + q * NN;
      mo.cols[mo.nq] = oc;
      ++mo.nq;
    }
    if (mo.nq == 0) continue;
    if (two) {
      // X3 holds one slot of n * cblk doubles per output
      const long slot = (long)n * cblk;
      y_inverse(m, X2, mo, X3, slot, yout);
      HM_LAUNCH_CHECK();
      mo.in_stride = slot;
      x_inverse(m, X3, mo, false, ldo, Nyo, xout, yout);
    } else {
      mo.in_stride = 0;
      x_inverse(m, Xh, mo, true, ldo, 1, xout, yout);
    }
    HM_LAUNCH_CHECK();
  }
  // The nugget tau2 I acts row by row, so it is added to the value output here rather
  // than as a mode multiplier: through the transforms its rounding (relative to the
  // largest entry of a column) would swamp the small far-field products the sketches
  // sample.  An input confined to one side of a split and an output wanted on the
  // other side get no nugget term at all.
  if (!m->uniform) {
    // the transforms write grid points only: the padding rows of the outputs are zero
    double* outs0[3] = {outK, outKap, outAlp};
    for (int q = 0; q < 3; ++q)
      if (outs0[q] && ocols[q] > 0) {
        hipLaunchKernelGGL(k_zero_pad_rows, dim3(ceil_div((long)n * ocols[q], 256)), dim3(256), 0, m->stream,
                           outs0[q], ldo, m->d_perm, n, ocols[q]);
        HM_LAUNCH_CHECK();
      }
  }
  HM_CHECK(add_nugget(m, theta, X, ldx, outK, cK, ldo, in_sel, out_sel));
  if (pf) {
    // bytes: each pass reads and writes its n x c block once (compact where the maps halve it), plus S
    const double frac_in = (double)Kx * Nyi / NN, frac_out = (double)Mx * Nyo / NN;
    const double passes = (two ? 1.0 + 1.0 : 1.0) * (0.5 + 0.5 * frac_in) + nout * (two ? 2.0 : 1.0) * 0.5 * (1.0 + frac_out);
    prof_end(m, PF_DST, per_col * c, passes * 16.0 * n * (double)c + 8.0 * N * (double)N);
  }
  return HM_OK;
}

hm_status kapply_multi(Model* m, const double* theta, const double* X, int ldx, int c, double* outK, int cK,
                       double* outKap, int cKap, double* outAlp, int cAlp, int ldo, LeafSel in_sel,
                       LeafSel out_sel) {
  return kapply_core(m, m->d_ws, m->cmax, theta, X, ldx, c, outK, cK, outKap, cKap, outAlp, cAlp, ldo, in_sel,
                     out_sel);
}

hm_status kapply_ws(Model* m, double* ws, int cblk, const double* theta, const double* X, int ldx, int c,
                    double* outK, double* outKap, double* outAlp, int ldo) {
  if (cblk < 1) {
    set_error("kapply: the scratch holds no column block");
    return HM_E_INVAL;
  }
  return kapply_core(m, ws, cblk, theta, X, ldx, c, outK, c, outKap, c, outAlp, c, ldo, sel_all(), sel_all());
}

hm_status kapply_sel(Model* m, const double* theta, const double* X, int ldx, int c, double* outK,
                     double* outKap, double* outAlp, int ldo, LeafSel in_sel, LeafSel out_sel) {
  return kapply_multi(m, theta, X, ldx, c, outK, c, outKap, c, outAlp, c, ldo, in_sel, out_sel);
}

hm_status kapply(Model* m, const double* theta, const double* X, int ldx, int c, double* outK,
                 double* outKap, double* outAlp, int ldo) {
  return kapply_sel(m, theta, X, ldx, c, outK, outKap, outAlp, ldo, sel_all(), sel_all());
}

TreeIdx make_tree_idx(int dim, int N, int levels) {
  TreeIdx t{};
  t.two = (dim == 2);
  if (!t.two) return t;
  const int cx = (levels + 1) / 2, cy = levels / 2;   // x splits first
  t.wl = N >> cx;
  t.hl = N >> cy;
  t.nl = t.wl * t.hl;
  t.sx = (levels % 2) ? 0 : 1;   // the last split is x when levels is odd
  t.sy = 1 - t.sx;
  t.mx = recip32(t.wl);
  t.my = recip32(t.hl);
  return t;
}

hm_status model_tables(Model* m) {
  m->tix = make_tree_idx(m->dim, m->N, m->levels);
  m->tix.N = m->N;
  const int n = m->n, N = m->N;
  if (m->uniform) {
    hipLaunchKernelGGL(k_perm, dim3(ceil_div(n, 256)), dim3(256), 0, m->stream, m->d_perm, m->d_iperm, n, N,
                       m->dim, m->levels, m->nl);
    HM_LAUNCH_CHECK();
  } else {
    m->tix.tab = m->d_iperm;   // tables uploaded by the model's creator
  }
  hipLaunchKernelGGL(k_tables, dim3(ceil_div((long)N * N, 256)), dim3(256), 0, m->stream, m->d_dst, m->d_mu, N,
                     m->dim, m->h);
  HM_LAUNCH_CHECK();
  if (m->d_dsth) {
    hipLaunchKernelGGL(k_tables_half, dim3(ceil_div((long)N * N, 256)), dim3(256), 0, m->stream, m->d_dsth, N);
    HM_LAUNCH_CHECK();
  }
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

// wmode[0..3] += (sigma2 <Yb, K_op X>, sigma2 <Yb, d0 K_op X>, sigma2 <Yb, d1 K_op X>, <Yb, X>)
// and, nq = 5, wmode[4] += <Yb, X> over the second variable's rows (bivariate model)
__global__ void k_accum(double* w, const double* d, double s, int nq) {
  const int q = threadIdx.x;
  if (q < nq) w[q] += (q < 3 ? s : 1.0) * d[q];
}
// Xs[i + j nr] = X[i + j nr] on the rows i >= split, else 0
__global__ void k_rows_from(double* Xs, const double* X, int nr, long split, int c) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)nr * c) return;
  Xs[e] = (e % nr) >= split ? X[e] : 0.0;
}

// columns of a tree-ordered block gathered into the operator's point order (ld n_real)
hm_status kvjp_gather(Model* m, const double* X, int ldx, double* Xn, int c) {
  hipLaunchKernelGGL(k_gather_nat, dim3(ceil_div((long)m->n_real * c, 256)), dim3(256), 0, m->stream, X, (long)ldx, Xn,
                     m->d_iperm, m->n_real, c);
  HM_LAUNCH_CHECK();
  return HM_OK;
}

// For an operator model the vector-Jacobian product has no mode structure: every
// parameter's term <Ybar, dK/dtheta_j X> is formed from the operator's derivative
// products (three operator applications per column block).
static hm_status kvjp_op(Model* m, const double* theta, const double* X, int ldx, const double* Yb, int ldb, int c,
                         double* wmode) {
  const int n = m->n, nr = m->n_real, cblk = m->cmax;
  double* Xn = m->d_ws;
  double* Bn = m->d_ws + (long)n * cblk;
  double* Yq[3] = {m->d_ws + 2L * n * cblk, m->d_ws + 3L * n * cblk, m->d_ws + 4L * n * cblk};
  for (int c0 = 0; c0 < c; c0 += cblk) {
    const int cc = std::min(cblk, c - c0);
    const long cnt = (long)nr * cc;
    hipLaunchKernelGGL(k_gather_nat, dim3(ceil_div(cnt, 256)), dim3(256), 0, m->stream, X + (long)c0 * ldx, (long)ldx,
                       Xn, m->d_iperm, nr, cc);
    HM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_gather_nat, dim3(ceil_div(cnt, 256)), dim3(256), 0, m->stream, Yb + (long)c0 * ldb,
                       (long)ldb, Bn, m->d_iperm, nr, cc);
    HM_LAUNCH_CHECK();
    for (int q = 0; q < 3; ++q) HM_CHECK(op_call(m, q, theta, Xn, cc, Yq[q]));
    const double* A[1] = {Bn};
    const double* B[4] = {Yq[0], Yq[1], Yq[2], Xn};
    double* out = m->d_opws + 1024 * 16;
    HM_CHECK(dots(m, A, 1, B, 4, cnt, out, m->d_opws));
    const int nq = m->nvars == 2 ? 5 : 4;
    if (nq == 5) {
      // the second variable's rows of X (in Yq[0], read above) for its nugget's sum
      hipLaunchKernelGGL(k_rows_from, dim3(ceil_div(cnt, 256)), dim3(256), 0, m->stream, Yq[0], Xn, nr, m->nsplit,
                         cc);
      HM_LAUNCH_CHECK();
      const double* B2[1] = {Yq[0]};
      HM_CHECK(dots(m, A, 1, B2, 1, cnt, out + 4, m->d_opws));
    }
    hipLaunchKernelGGL(k_accum, dim3(1), dim3(64), 0, m->stream, wmode, out, theta[3], nq);
    HM_LAUNCH_CHECK();
  }
  return HM_OK;
}

hm_status kvjp(Model* m, const double* theta, const double* X, int ldx, const double* Yb, int ldb, int c,
               double* wmode) {
  if (c <= 0) return HM_OK;
  if (m->op_vjp) return m->op_vjp(m, theta, X, ldx, Yb, ldb, c, wmode);
  if (m->op) return kvjp_op(m, theta, X, ldx, Yb, ldb, c, wmode);
  HM_CHECK(ensure_scale(m, theta));
  const int n = m->n, N = m->N;
  const int Ny = (m->dim == 2) ? N : 1;
  const long NN = (long)N * Ny;
  double* W0 = m->d_ws;
  double* W1 = m->d_ws + (long)n * m->cmax;
  double* W2 = m->d_ws + 2L * n * m->cmax;
  const AxisMap id = axis_map(0, 0);
  for (int c0 = 0; c0 < c; c0 += m->cmax) {
    const int cc = std::min(m->cmax, c - c0);
    const double* Xc = X + (long)c0 * ldx;
    const double* Bc = Yb + (long)c0 * ldb;
    const double *ha, *hb;
    if (m->dim == 2) {
      x_forward(m, Xc, ldx, W0, cc, Ny, id, id);
      HM_LAUNCH_CHECK();
      y_forward(m, W0, W1, cc, id);
      HM_LAUNCH_CHECK();
      x_forward(m, Bc, ldb, W2, cc, Ny, id, id);
      HM_LAUNCH_CHECK();
      y_forward(m, W2, W0, cc, id);
      HM_LAUNCH_CHECK();
      ha = W1;
      hb = W0;
    } else {
      x_forward(m, Xc, ldx, W0, cc, Ny, id, id);
      HM_LAUNCH_CHECK();
      x_forward(m, Bc, ldb, W1, cc, Ny, id, id);
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
