// Exact traces for the score and the Fisher information (Sec. 4.2-4.3, App. B).
//
// With the factors of K~ (hm_factor.h) the inverse has the closed form
//   K~^{-1} = Dbar^{-1} - sum_P G_P N_P G_P^T,   G_P = diag(G_a, G_b) on P's rows,
// (unrolling K~_P^{-1} = (I - U_P N_P J V_P^T) diag(K~_a^{-1}, K~_b^{-1}) over the tree), so for
// any symmetric HODLR B on the same tree (App. B: products of HODLR matrices
// written as a HODLR part plus block-diagonal low-rank terms, whose traces are
// sums over leaves and nodes):
//   tr(K~^{-1} B) = sum_L <D_L^{-1}, B_L> - sum_P <N_P, G_P^T B_PP G_P>
// with G_P^T B_PP G_P = [[G_a^T Xi_a, X_ab], [X_ab^T, G_b^T Xi_b]], Xi_c = B_cc G_c,
// X_ab = G_a^T B_ab G_b.  No recompression and no stochastic estimator: exact.
// The Fisher entry (Sec. 4.3, eq. "fisher info approximated") is the derivative
// of that formula along K~_i with B = K~_j held fixed:
//   I_ij = -1/2 d_i tr(K~^{-1} K~_j)
//        = 1/2 sum_L tr(Y^i_L Y^j_L) - 1/2 sum_P <N_P dS^i_P N_P, Psi^j_P>
//          + sum_P tr(N_P dG_P^{iT} B^j_PP G_P),
// Y^i = Dbar^{-1} dD^i, dS^i_c = d(F_c^T G_c), dG^i_c = K~_c^{-1} (dF^i_c - Xi^i_c);
// the last sum is expanded into panel-wide inner products (see fim_terms).
// Every pair (i, j) is computed on its own, so symmetry of the result is a check.
#include <cmath>

#include "hm_build.h"
#include "hm_factor.h"
#include "hm_internal.h"
#include "hm_trace.h"

namespace hm {

// ---------------------------------------------------------------------------
// small element-wise kernels
// ---------------------------------------------------------------------------
__global__ void k_axpby(double* y, const double* x, long cnt, double a, double b) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < cnt) y[e] = a * x[e] + b * y[e];
}
__global__ void k_lin2(double* out, const double* x1, const double* x2, long cnt, double a1, double a2) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < cnt) out[e] = a1 * x1[e] + (x2 ? a2 * x2[e] : 0.0);
}
// leaf-major: out_L = a * A_L + b * I
__global__ void k_leaf_affine(double* out, const double* A, int nl, long cnt, double a, double b) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= cnt) return;
  int le = (int)(e % ((long)nl * nl));
  double v = (A ? a * A[e] : 0.0);
  if (le % nl == le / nl) v += b;
  out[e] = v;
}

// Per-row coefficients of the bivariate model's nugget structure: row t of the tree
// order takes c0 (first variable), c1 (second variable: natural index >= split) or 0
// (padding row).
__device__ __forceinline__ double row_coef(const int* perm, long t, long split, double c0, double c1) {
  const int g = perm[t];
  return g < 0 ? 0.0 : (g >= split ? c1 : c0);
}
// panel set (ld n): out[t + j n] = coef(t) in[t + j n]
__global__ void k_rows_coef(double* out, const double* in, long n, long cnt, const int* perm, long split, double c0,
                            double c1) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < cnt) out[e] = row_coef(perm, e % n, split, c0, c1) * in[e];
}
// leaf-major: out_L = a A_L + diag(coef(rows of L))   (A may be null)
__global__ void k_leaf_diag_coef(double* out, const double* A, int nl, long cnt, const int* perm, long split,
                                 double a, double c0, double c1) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= cnt) return;
  const long ls = (long)nl * nl, L = e / ls;
  const int le = (int)(e % ls), i = le % nl, j = le / nl;
  double v = A ? a * A[e] : 0.0;
  if (i == j) v += row_coef(perm, L * nl + i, split, c0, c1);
  out[e] = v;
}
// leaf-major: out_L = a Dinv_L diag(coef(columns of L)) + b I on the real rows
__global__ void k_leaf_col_coef(double* out, const double* Dinv, int nl, long cnt, const int* perm, long split,
                                double a, double c0, double c1, double b) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= cnt) return;
  const long ls = (long)nl * nl, L = e / ls;
  const int le = (int)(e % ls), i = le % nl, j = le / nl;
  double v = a * Dinv[e] * row_coef(perm, L * nl + j, split, c0, c1);
  if (i == j && perm[L * nl + i] >= 0) v += b;
  out[e] = v;
}

static hm_status lin2(Model* m, double* out, const double* x1, const double* x2, long cnt, double a1, double a2) {
  hipLaunchKernelGGL(k_lin2, dim3(ceil_div(cnt, 256)), dim3(256), 0, m->stream, out, x1, x2, cnt, a1, a2);
  HM_LAUNCH_CHECK();
  return HM_OK;
}
static hm_status leaf_affine(Model* m, double* out, const double* A, double a, double b) {
  long cnt = (long)m->nleaves * m->nl * m->nl;
  hipLaunchKernelGGL(k_leaf_affine, dim3(ceil_div(cnt, 256)), dim3(256), 0, m->stream, out, A, m->nl, cnt, a, b);
  HM_LAUNCH_CHECK();
  return HM_OK;
}

// ---------------------------------------------------------------------------
// dot products of long vectors: out[i*nb + j] = sum_e A_i[e] B_j[e]
// (two phases, deterministic order)
// ---------------------------------------------------------------------------
struct DotArgs {
  const double* A[4];
  const double* B[4];
  int na, nb;
  long len;
};
constexpr int DOT_BLOCKS = 1024;

__global__ void __launch_bounds__(256) k_dots_partial(DotArgs a, double* partial) {
  __shared__ double red[256];
  double acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.0;
  // Four grid strides per step, with loads free of branches so that all of them are in
  // flight together: operands past na / nb read the first one, elements past len read
  // the step's first element, and both are zeroed at use.
  constexpr int U = 4;
  const double* Ap[4];
  const double* Bp[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    Ap[i] = a.A[i < a.na ? i : 0];
    Bp[i] = a.B[i < a.nb ? i : 0];
  }
  const long stride = (long)gridDim.x * blockDim.x;
  for (long e0 = (long)blockIdx.x * blockDim.x + threadIdx.x; e0 < a.len; e0 += U * stride) {
    double av[U][4], bv[U][4];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long e = e0 + u * stride;
      const long ec = e < a.len ? e : e0;
#pragma unroll
      for (int i = 0; i < 4; ++i) av[u][i] = Ap[i][ec];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[u][j] = Bp[j][ec];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool ok = e0 + u * stride < a.len;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const double x = (ok && i < a.na) ? av[u][i] : 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i * 4 + j] += x * bv[u][j];
      }
    }
  }
  for (int q = 0; q < a.na * a.nb; ++q) {
    int i = q / a.nb, j = q % a.nb;
    red[threadIdx.x] = acc[i * 4 + j];
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
      if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[(long)blockIdx.x * 16 + q] = red[0];
    __syncthreads();
  }
}
__global__ void k_dots_final(const double* partial, int nblocks, int nq, double* out) {
  __shared__ double red[256];
  const int q = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) s += partial[(long)b * 16 + q];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[q] = red[0];
}

hm_status dots(Model* m, const double* const* A, int na, const double* const* B, int nb, long len, double* out,
               double* partial) {
  DotArgs a{};
  for (int i = 0; i < na; ++i) a.A[i] = A[i];
  for (int j = 0; j < nb; ++j) a.B[j] = B[j];
  a.na = na;
  a.nb = nb;
  a.len = len;
  int nblk = (int)std::min<long>(DOT_BLOCKS, std::max<long>(1, ceil_div(len, 256)));
  hipLaunchKernelGGL(k_dots_partial, dim3(nblk), dim3(256), 0, m->stream, a, partial);
  HM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_dots_final, dim3(na * nb), dim3(256), 0, m->stream, partial, nblk, na * nb, out);
  HM_LAUNCH_CHECK();
  return HM_OK;
}

// Pairwise traces of leaf-major blocks: out[i nb + j] = sum_L tr(A_i[L] B_j[L]) =
// sum_L sum_{a,b} A_i[L](a, b) B_j[L](b, a).  One 32 x 32 tile (L, a0, b0) per step: the
// B_j tiles at the transposed position go through LDS, so both operands are read in
// 256-byte column runs.  Partial sums as in k_dots_partial.  sym (B_j = A_j for every j):
// the tile pair (a0, b0), (b0, a0) is visited once, a0 <= b0, since the pair's second tile
// contributes to (i, j) what the first contributes to (j, i); every block is read once.
constexpr int LT = 32;
__global__ void __launch_bounds__(256) k_dots_leafT_partial(DotArgs a, int nl, int nleaves, int sym,
                                                            double* partial) {
  __shared__ double red[256];
  __shared__ double Bt[4][LT][LT + 1];
  double acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.0;
  const int tpl = (nl + LT - 1) / LT;             // tiles per leaf side
  const int tpp = sym ? tpl * (tpl + 1) / 2 : tpl * tpl;   // tiles (pairs) per leaf
  const long ntiles = (long)nleaves * tpp;
  const int tx = threadIdx.x % LT, ty = threadIdx.x / LT;   // 32 x 8 threads
  const long ls = (long)nl * nl;
  // operands past na / nb read the first one (zeroed at use), so the loads of a step
  // carry no branches and all of them, A's and B's, are in flight together
  const double* Ap[4];
  const double* Bp[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    Ap[i] = a.A[i < a.na ? i : 0];
    Bp[i] = a.B[i < a.nb ? i : 0];
  }
  constexpr int RS = LT / 8;   // rows of a tile per thread
  for (long t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int L = (int)(t / tpp);
    int rem = (int)(t % tpp), ta, tb;
    if (sym) {   // pairs ta <= tb, ordered by tb
      tb = 0;
      while (rem > tb) {
        rem -= tb + 1;
        ++tb;
      }
      ta = rem;
    } else {
      ta = rem % tpl;
      tb = rem / tpl;
    }
    const int a0 = ta * LT, b0 = tb * LT;
    const bool twice = sym && ta != tb;
    const long lb = L * ls;
    double bt[4][RS], at[4][RS];
    bool okb[RS], oka[RS];
#pragma unroll
    for (int s = 0; s < RS; ++s) {
      const int r = ty + 8 * s;
      // B_j(b0 + tx, a0 + r), to Bt[j][tx][r]
      const int row = b0 + tx, col = a0 + r;
      okb[s] = row < nl && col < nl;
      const long ob = lb + (okb[s] ? row + (long)col * nl : 0);
#pragma unroll
      for (int j = 0; j < 4; ++j) bt[j][s] = Bp[j][ob];
      // A_i(a0 + tx, b0 + r), which pairs with B_j(b0 + r, a0 + tx) = Bt[j][r][tx]
      const int ra = a0 + tx, ca = b0 + r;
      oka[s] = ra < nl && ca < nl;
      const long oa = lb + (oka[s] ? ra + (long)ca * nl : 0);
#pragma unroll
      for (int i = 0; i < 4; ++i) at[i][s] = Ap[i][oa];
    }
#pragma unroll
    for (int s = 0; s < RS; ++s)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (j < a.nb) Bt[j][tx][ty + 8 * s] = okb[s] ? bt[j][s] : 0.0;
    __syncthreads();
#pragma unroll
    for (int s = 0; s < RS; ++s) {
      double av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = (oka[s] && i < a.na) ? at[i][s] : 0.0;
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = (j < a.nb) ? Bt[j][ty + 8 * s][tx] : 0.0;
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i * 4 + j] += av[i] * bv[j] + (twice ? av[j] * bv[i] : 0.0);
    }
    __syncthreads();
  }
  for (int q = 0; q < a.na * a.nb; ++q) {
    int i = q / a.nb, j = q % a.nb;
    red[threadIdx.x] = acc[i * 4 + j];
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
      if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[(long)blockIdx.x * 16 + q] = red[0];
    __syncthreads();
  }
}
hm_status dots_leafT(Model* m, const double* const* A, int na, const double* const* B, int nb, double* out,
                     double* partial) {
  DotArgs a{};
  for (int i = 0; i < na; ++i) a.A[i] = A[i];
  for (int j = 0; j < nb; ++j) a.B[j] = B[j];
  a.na = na;
  a.nb = nb;
  bool sym = na == nb;
  for (int i = 0; i < na && sym; ++i) sym = A[i] == B[i];
  const int tpl = ceil_div(m->nl, LT);
  const long ntiles = (long)m->nleaves * (sym ? tpl * (tpl + 1) / 2 : tpl * tpl);
  const int nblk = (int)std::min<long>(DOT_BLOCKS, std::max<long>(1, ntiles));
  hipLaunchKernelGGL(k_dots_leafT_partial, dim3(nblk), dim3(256), 0, m->stream, a, m->nl, m->nleaves, sym ? 1 : 0,
                     partial);
  HM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_dots_final, dim3(na * nb), dim3(256), 0, m->stream, partial, nblk, na * nb, out);
  HM_LAUNCH_CHECK();
  return HM_OK;
}

// sum of the diagonals of the leaf-major blocks; or a plain sum (stride 1) when nl==0
__global__ void k_sum_partial(const double* x, long len, int nl, double* partial) {
  __shared__ double red[256];
  double s = 0.0;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < len; e += (long)gridDim.x * blockDim.x) {
    if (nl > 0) {
      long L = e / nl, i = e % nl;
      s += x[L * nl * nl + i + i * nl];
    } else {
      s += x[e];
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(long)blockIdx.x * 16] = red[0];
}
hm_status sum_scalar(Model* m, const double* x, long len, int diag_nl, double* out, double* partial) {
  int nblk = (int)std::min<long>(DOT_BLOCKS, std::max<long>(1, ceil_div(len, 256)));
  hipLaunchKernelGGL(k_sum_partial, dim3(nblk), dim3(256), 0, m->stream, x, len, diag_nl, partial);
  HM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_dots_final, dim3(1), dim3(256), 0, m->stream, partial, nblk, 1, out);
  HM_LAUNCH_CHECK();
  return HM_OK;
}

// ---------------------------------------------------------------------------
// Per-node small products.  Every internal node P (heap 0..nint-1, children
// a = 2P+1, b = 2P+2) is one batch entry of a strided batched GEMM, so each
// product is a single launch over the whole tree.
//   N_P blocks: N11 = N[0:k,0:k] (at N), N12 = N[0:k,k:2k] (at N + k*m),
//               N21 = N[k:2k,0:k] (at N + k), N22 (at N + k + k*m); m = 2k, ld m.
// ---------------------------------------------------------------------------
// out_a = N11, out_b = N22 (copies); all internal nodes
__global__ void k_node_diag(const double* Nn, double* Ncc, int kc, int nint) {
  const long s2 = (long)kc * kc;
  const int m2 = 2 * kc;
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nint * s2) return;
  int P = (int)(e / s2);
  int r = (int)(e % s2), i = r % kc, j = r / kc;
  const double* N = Nn + (long)P * m2 * m2;
  Ncc[(2L * P + 1) * s2 + r] = N[i + (long)j * m2];
  Ncc[(2L * P + 2) * s2 + r] = N[(kc + i) + (long)(kc + j) * m2];
}

// PsiP = [[Psi_a, X_P], [X_P^T, Psi_b]] for all internal nodes
__global__ void k_node_psi_assemble(const double* Psi, const double* X, double* PsiP, int kc, int nint) {
  const long s2 = (long)kc * kc;
  const int m2 = 2 * kc;
  const long ms = (long)m2 * m2;
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nint * ms) return;
  int P = (int)(e / ms);
  int r = (int)(e % ms), i = r % m2, j = r / m2;
  double v;
  if (i < kc && j < kc) v = Psi[(2L * P + 1) * s2 + i + (long)j * kc];
  else if (i >= kc && j >= kc) v = Psi[(2L * P + 2) * s2 + (i - kc) + (long)(j - kc) * kc];
  else if (i < kc) v = X[P * s2 + i + (long)(j - kc) * kc];
  else v = X[P * s2 + j + (long)(i - kc) * kc];
  PsiP[e] = v;
}

// dS_c = E_c + W_c^T for all non-root nodes
__global__ void k_node_dS(const double* E, const double* W, double* dS, int kc, long nodes) {
  const long s2 = (long)kc * kc;
  long e = s2 + (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nodes * s2) return;
  long c = e / s2;
  int r = (int)(e % s2), i = r % kc, j = r / kc;
  dS[e] = E[e] + W[c * s2 + j + (long)i * kc];
}

hm_status node_prep(FactorCtx& f) {
  Model* m = f.m;
  const int kc = f.kc, m2 = 2 * kc;
  const long s2 = (long)kc * kc, ms = (long)m2 * m2;
  const int nint = (1 << m->levels) - 1;
  hipLaunchKernelGGL(k_node_diag, dim3(ceil_div(nint * s2, 256)), dim3(256), 0, m->stream, f.Nn, f.Ncc, kc, nint);
  HM_LAUNCH_CHECK();
  // Nx_a = N12 S_b,  Nx_b = N21 S_a
  HM_CHECK(gemm(m->stream, false, false, kc, kc, kc, 1.0, f.Nn + (long)kc * m2, m2, ms, f.Sn + 2 * s2, kc, 2 * s2,
                0.0, f.Nx + s2, kc, 2 * s2, nint));
  HM_CHECK(gemm(m->stream, false, false, kc, kc, kc, 1.0, f.Nn + kc, m2, ms, f.Sn + s2, kc, 2 * s2, 0.0,
                f.Nx + 2 * s2, kc, 2 * s2, nint));
  return HM_OK;
}

// PsiP^j for every internal node (X_ab = E_a^T S_b + S_a E_b)
hm_status node_psi(FactorCtx& f, ParamBufs& pb, double* xtmp) {
  Model* m = f.m;
  const int kc = f.kc;
  const long s2 = (long)kc * kc, ms = 4 * s2;
  const int nint = (1 << m->levels) - 1;
  HM_CHECK(gemm(m->stream, true, false, kc, kc, kc, 1.0, pb.E + s2, kc, 2 * s2, f.Sn + 2 * s2, kc, 2 * s2, 0.0,
                xtmp, kc, s2, nint));
  HM_CHECK(gemm(m->stream, false, false, kc, kc, kc, 1.0, f.Sn + s2, kc, 2 * s2, pb.E + 2 * s2, kc, 2 * s2, 1.0,
                xtmp, kc, s2, nint));
  hipLaunchKernelGGL(k_node_psi_assemble, dim3(ceil_div(nint * ms, 256)), dim3(256), 0, m->stream, pb.Psi, xtmp,
                     pb.PsiP, kc, nint);
  HM_LAUNCH_CHECK();
  return HM_OK;
}

// Lam^j = N diag(dS_a, dS_b) N and Vt^j for every internal node
hm_status node_lam(FactorCtx& f, ParamBufs& pb, double* tbuf, double* dsbuf) {
  Model* m = f.m;
  const int kc = f.kc, m2 = 2 * kc;
  const long s2 = (long)kc * kc, ms = (long)m2 * m2;
  const int nint = (1 << m->levels) - 1;
  const long nodes = (2L << m->levels) - 1;
  hipLaunchKernelGGL(k_node_dS, dim3(ceil_div((nodes - 1) * s2, 256)), dim3(256), 0, m->stream, pb.E, pb.W, dsbuf,
                     kc, nodes);
  HM_LAUNCH_CHECK();
  // T = [N[:,0:k] dS_a, N[:,k:2k] dS_b]: one batch over (P, half h), b = 2P + h, whose
  // operands sit at uniform strides: the column half of N_P and of T at b (2 k^2) (a
  // half is k columns of 2k rows), dS of child 2P + 1 + h at (b + 1) k^2
  HM_CHECK(gemm(m->stream, false, false, m2, kc, kc, 1.0, f.Nn, m2, 2 * s2, dsbuf + s2, kc, s2, 0.0, tbuf, m2,
                2 * s2, 2 * nint));
  HM_CHECK(gemm(m->stream, false, false, m2, m2, m2, 1.0, tbuf, m2, ms, f.Nn, m2, ms, 0.0, pb.Lam, m2, ms, nint));
  // Vt_a = W_b^T N21,  Vt_b = W_a^T N12
  HM_CHECK(gemm(m->stream, true, false, kc, kc, kc, 1.0, pb.W + 2 * s2, kc, 2 * s2, f.Nn + kc, m2, ms, 0.0,
                pb.Vt + s2, kc, 2 * s2, nint));
  HM_CHECK(gemm(m->stream, true, false, kc, kc, kc, 1.0, pb.W + s2, kc, 2 * s2, f.Nn + (long)kc * m2, m2, ms, 0.0,
                pb.Vt + 2 * s2, kc, 2 * s2, nint));
  return HM_OK;
}

// ---------------------------------------------------------------------------
// per-parameter work
// ---------------------------------------------------------------------------
hm_status param_prepare(FactorCtx& f, ParamBufs& pb, const double* theta, const double* tF_prefix,
                        const double* GtG) {
  Model* m = f.m;
  PrecScope prec(m, true);   // trace panels: FP32 (BF16 under policy 2) under the mixed policies
  const int n = m->n, kc = f.kc, levels = m->levels;
  const long pcnt = (long)n * levels * kc;
  const long s2 = (long)kc * kc;
  const long ncnt = ((2L << levels) - 2) * s2;   // per-node arrays, non-root nodes (from offset s2)
  const double tau2 = theta[2], sigma2 = theta[3];
  if (m->nvars == 2 && pb.kind >= 2) {
    // bivariate model: K~ = sigma2-scaled physics + diag(T), T = tau2_1 on the first
    // variable's rows, tau2_2 on the second's (M_v: the rows of variable v)
    const long lcnt = (long)m->nleaves * m->nl * m->nl;
    const long split = m->nsplit;
    const int* perm = m->d_perm;
    const dim3 gp(ceil_div(pcnt, 256)), gl(ceil_div(lcnt, 256));
    const ReduceJob rp{f.G, n, cs_block(kc), pb.Xi, n, cs_block(kc), 1, levels, pb.Psi, s2, sel_all()};
    if (pb.kind == 2 || pb.kind == 4) {
      // K~_tau2_v = M_v: no panels; dD = M_v, Xi = M_v G, Y = Dinv M_v, Psi = G^T M_v G, E = 0
      const double c0 = pb.kind == 2 ? 1.0 : 0.0, c1 = 1.0 - c0;
      HM_CHECK(fill(m, pb.dF, pcnt, 0.0));
      hipLaunchKernelGGL(k_leaf_diag_coef, gl, dim3(256), 0, m->stream, pb.dD, nullptr, m->nl, lcnt, perm, split, 0.0,
                         c0, c1);
      HM_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_rows_coef, gp, dim3(256), 0, m->stream, pb.Xi, f.G, (long)n, pcnt, perm, split, c0, c1);
      HM_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_leaf_col_coef, gl, dim3(256), 0, m->stream, pb.Y, f.Dinv, m->nl, lcnt, perm, split, 1.0, c0,
                         c1, 0.0);
      HM_LAUNCH_CHECK();
      HM_CHECK(fill(m, pb.E + s2, ncnt, 0.0));
      HM_CHECK(tree_reduce(m, rp));
      return HM_OK;
    }
    // K~_sigma2 = (K~ - T) / sigma2: dF = F / (2 sigma2), dD = (D - T) / sigma2,
    // Xi = (F - T G) / sigma2, Y = (I - Dinv T) / sigma2, E = S / (2 sigma2),
    // Psi = (S - G^T T G) / sigma2
    const double t1 = theta[2], t2 = theta[4];
    HM_CHECK(lin2(m, pb.dF, f.F, nullptr, pcnt, 0.5 / sigma2, 0.0));
    hipLaunchKernelGGL(k_leaf_diag_coef, gl, dim3(256), 0, m->stream, pb.dD, f.D, m->nl, lcnt, perm, split,
                       1.0 / sigma2, -t1 / sigma2, -t2 / sigma2);
    HM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_rows_coef, gp, dim3(256), 0, m->stream, pb.Xi, f.G, (long)n, pcnt, perm, split, t1, t2);
    HM_LAUNCH_CHECK();
    HM_CHECK(tree_reduce(m, rp));                                   // G^T T G
    HM_CHECK(lin2(m, pb.Psi + s2, f.Sn + s2, pb.Psi + s2, ncnt, 1.0 / sigma2, -1.0 / sigma2));
    HM_CHECK(lin2(m, pb.Xi, f.F, pb.Xi, pcnt, 1.0 / sigma2, -1.0 / sigma2));
    hipLaunchKernelGGL(k_leaf_col_coef, gl, dim3(256), 0, m->stream, pb.Y, f.Dinv, m->nl, lcnt, perm, split,
                       -1.0 / sigma2, t1, t2, 1.0 / sigma2);
    HM_LAUNCH_CHECK();
    HM_CHECK(lin2(m, pb.E + s2, f.Sn + s2, nullptr, ncnt, 0.5 / sigma2, 0.0));
    HM_CHECK(leaf_pad(m, pb.dD, 0.0));
    return HM_OK;
  }
  if (pb.kind == 2) {
    // K~_tau2 = I: no panels, identity leaves.  Xi = G, Y = Dinv and Psi = G^T G are
    // aliases set at creation; E = dF^T G = 0.
    HM_CHECK(fill(m, pb.dF, pcnt, 0.0));
    HM_CHECK(leaf_affine(m, pb.dD, nullptr, 0.0, 1.0));
    HM_CHECK(fill(m, pb.E + s2, ncnt, 0.0));
    if (!m->uniform) {
      // K~_tau2 is the identity on the real rows only; Y = Dinv restricted to them
      HM_CHECK(leaf_pad(m, pb.dD, 0.0));
      HM_CHECK(leaf_affine(m, pb.Y, f.Dinv, 1.0, 0.0));
      HM_CHECK(leaf_pad(m, pb.Y, 0.0));
    }
    return HM_OK;
  }
  if (pb.kind == 3) {
    // K~_sigma2 = (K~ - tau2 I)/sigma2: dF = F/(2 sigma2), dD = (D - tau2 I)/sigma2,
    // Xi = (F - tau2 G)/sigma2, Y = Dinv dD = (I - tau2 Dinv)/sigma2,
    // E = dF^T G = S/(2 sigma2), Psi = G^T Xi = (S - tau2 G^T G)/sigma2  (S = F^T G, symmetric)
    HM_CHECK(lin2(m, pb.dF, f.F, nullptr, pcnt, 0.5 / sigma2, 0.0));
    HM_CHECK(leaf_affine(m, pb.dD, f.D, 1.0 / sigma2, -tau2 / sigma2));
    HM_CHECK(lin2(m, pb.Xi, f.F, f.G, pcnt, 1.0 / sigma2, -tau2 / sigma2));
    HM_CHECK(leaf_affine(m, pb.Y, f.Dinv, -tau2 / sigma2, 1.0 / sigma2));
    HM_CHECK(lin2(m, pb.E + s2, f.Sn + s2, nullptr, ncnt, 0.5 / sigma2, 0.0));
    HM_CHECK(lin2(m, pb.Psi + s2, f.Sn + s2, GtG + s2, ncnt, 1.0 / sigma2, -tau2 / sigma2));
    HM_CHECK(leaf_pad(m, pb.dD, 0.0));
    HM_CHECK(leaf_pad(m, pb.Y, 0.0));
    return HM_OK;
  }
  // Xi_c = B_cc G_c: leaves plus every sibling pair strictly inside c
  HM_CHECK(leaf_gemm(m, pb.dD, f.G, n, pb.Xi, n, levels * kc, 1.0, 0.0, 0, m->nleaves));
  if (levels >= 2) {
    const long ts = (long)kc * (levels - 1) * kc;
    ReduceJob rd{pb.dF, n, cs_block(kc), f.G, n, cs_prefix(kc), 2, levels, f.nU, ts, sel_all()};
    HM_CHECK(tree_reduce(m, rd));
    ExpandJob e{pb.dF, n, cs_block(kc), pb.Xi, n, cs_prefix(kc), tF_prefix, ts, kc, 1, 0, 2, levels, 1.0, 1.0,
                sel_all()};
    e.A2 = f.F;
    e.T2 = f.nU;
    e.alpha2 = 1.0;
    HM_CHECK(tree_expand(m, e));
  }
  // leaf products Y = Dinv dD (dD Dinv = Y^T: both factors are symmetric, so the
  // Fisher's leaf term tr(Dinv dD_i Dinv dD_j) is a transposed dot of Y_i and Y_j)
  const int nl = m->nl;
  const long ls = (long)nl * nl;
  HM_CHECK(gemm(m->stream, false, false, nl, nl, nl, 1.0, f.Dinv, nl, ls, pb.dD, nl, ls, 0.0, pb.Y, nl, ls,
                m->nleaves));
  // E_c = dF_c^T G_c,  Psi_c = G_c^T Xi_c  (all non-root nodes)
  const ReduceJob rj[2] = {
      ReduceJob{pb.dF, n, cs_block(kc), f.G, n, cs_block(kc), 1, levels, pb.E, s2, sel_all()},
      ReduceJob{f.G, n, cs_block(kc), pb.Xi, n, cs_block(kc), 1, levels, pb.Psi, s2, sel_all()}};
  HM_CHECK(tree_reduce_multi(m, rj, 2));   // independent: one launch
  return HM_OK;
}

// sigma2 from tau2: with H_c = K~_c^{-1} G_c, dG_tau2 = -H and
//   dG_sigma2 = K~_c^{-1}(F/(2 sigma2) - (F - tau2 G)/sigma2) = -G/(2 sigma2) - (tau2/sigma2) dG_tau2,
//   W_sigma2 = dG_sigma2^T F = -S/(2 sigma2) - (tau2/sigma2) W_tau2.
hm_status scale_sweep(FactorCtx& f, ParamBufs& ps, const ParamBufs& pt, const double* theta) {
  Model* m = f.m;
  const int n = m->n, kc = f.kc, levels = m->levels;
  const long pcnt = (long)n * levels * kc;
  const long s2 = (long)kc * kc;
  const long ncnt = ((2L << levels) - 2) * s2;   // non-root nodes
  const double tau2 = theta[2], sigma2 = theta[3];
  HM_CHECK(lin2(m, ps.dG, f.G, pt.dG, pcnt, -0.5 / sigma2, -tau2 / sigma2));
  HM_CHECK(lin2(m, ps.W + s2, f.Sn + s2, pt.W + s2, ncnt, -0.5 / sigma2, -tau2 / sigma2));
  return HM_OK;
}

// dG_c = K~_c^{-1} (dF_c - Xi_c) for every non-root node c, all depths at once:
//   K~_c^{-1} X = Dbar_c^{-1} X - sum_{P in subtree(c)} G_P N_P G_P^T X.
hm_status tangent_sweep(FactorCtx& f, ParamBufs& pb) {
  Model* m = f.m;
  PrecScope prec(m, true);   // trace panels: FP32 (BF16 under policy 2) under the mixed policies
  const int n = m->n, kc = f.kc, levels = m->levels;
  const long pcnt = (long)n * levels * kc;
  double* R = f.tmp_panel;
  HM_CHECK(lin2(m, R, pb.dF, pb.Xi, pcnt, 1.0, -1.0));
  HM_CHECK(leaf_gemm(m, f.Dinv, R, n, pb.dG, n, levels * kc, 1.0, 0.0, 0, m->nleaves));
  if (levels >= 2) {
    const long ts = (long)kc * (levels - 1) * kc;
    const long us = 2L * kc * (levels - 1) * kc;
    ReduceJob r{f.G, n, cs_block(kc), R, n, cs_prefix(kc), 2, levels, f.nT, ts, sel_all()};
    HM_CHECK(tree_reduce(m, r));
    // U_P = N_P [T_a; T_b] for every depth 1..levels-1 at once (widths dP kc)
    HM_CHECK(node_apply_range(m, f.Nn, f.nT, ts, f.nU, us, kc, 0, kc, 1, levels - 1));
    ExpandJob e{f.G, n, cs_block(kc), pb.dG, n, cs_prefix(kc), f.nU, us, 2 * kc, 2, kc, 2, levels, -1.0, 1.0,
                sel_all()};
    HM_CHECK(tree_expand(m, e));
  }
  // W_c = dG_c^T F_c
  const long s2 = (long)kc * kc;
  ReduceJob rw{pb.dG, n, cs_block(kc), f.F, n, cs_block(kc), 1, levels, pb.W, s2, sel_all()};
  HM_CHECK(tree_reduce(m, rw));
  return HM_OK;
}

// Gh_c = dG_c N_P[c,c],  Hh_c = dG_c N_P[c,sib] S_sib
hm_status panel_products(FactorCtx& f, ParamBufs& pb) {
  Model* m = f.m;
  PrecScope prec(m, true);   // trace panels: FP32 (BF16 under policy 2) under the mixed policies
  const int n = m->n, kc = f.kc, levels = m->levels;
  const long s2 = (long)kc * kc;
  const ExpandJob ej[2] = {
      ExpandJob{pb.dG, n, cs_block(kc), pb.Gh, n, cs_block(kc), f.Ncc, s2, kc, 0, 0, 1, levels, 1.0, 0.0, sel_all()},
      ExpandJob{pb.dG, n, cs_block(kc), pb.Hh, n, cs_block(kc), f.Nx, s2, kc, 0, 0, 1, levels, 1.0, 0.0, sel_all()}};
  HM_CHECK(tree_expand_multi(m, ej, 2));   // independent: one launch
  return HM_OK;
}

}  // namespace hm
