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
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < a.len; e += (long)gridDim.x * blockDim.x) {
    double av[4], bv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) av[i] = (i < a.na) ? a.A[i][e] : 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) bv[j] = (j < a.nb) ? a.B[j][e] : 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i * 4 + j] += av[i] * bv[j];
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
  int q = threadIdx.x;
  if (q >= nq) return;
  double s = 0.0;
  for (int b = 0; b < nblocks; ++b) s += partial[(long)b * 16 + q];
  out[q] = s;
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
  hipLaunchKernelGGL(k_dots_final, dim3(1), dim3(64), 0, m->stream, partial, nblk, na * nb, out);
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
  hipLaunchKernelGGL(k_dots_final, dim3(1), dim3(64), 0, m->stream, partial, nblk, 1, out);
  HM_LAUNCH_CHECK();
  return HM_OK;
}

// ---------------------------------------------------------------------------
// per-node preparation: Ncc_c = N_P[c,c], Nx_c = N_P[c,sib] S_sib (children of P)
// ---------------------------------------------------------------------------
__global__ void k_node_prep(const double* Nn, const double* Sn, double* Ncc, double* Nx, int kc, int heap0) {
  const int P = heap0 + blockIdx.x;
  const int m2 = 2 * kc;
  const long s2 = (long)kc * kc;
  const double* N = Nn + (long)P * m2 * m2;
  const int a = 2 * P + 1, b = 2 * P + 2;
  for (int e = threadIdx.x; e < kc * kc; e += blockDim.x) {
    int i = e % kc, j = e / kc;
    Ncc[a * s2 + e] = N[i + (long)j * m2];
    Ncc[b * s2 + e] = N[(kc + i) + (long)(kc + j) * m2];
    double sa = 0.0, sb = 0.0;
    for (int l = 0; l < kc; ++l) {
      sa += N[i + (long)(kc + l) * m2] * Sn[b * s2 + l + (long)j * kc];      // N[a,b] S_b
      sb += N[(kc + i) + (long)l * m2] * Sn[a * s2 + l + (long)j * kc];      // N[b,a] S_a
    }
    Nx[a * s2 + e] = sa;
    Nx[b * s2 + e] = sb;
  }
}

// ---------------------------------------------------------------------------
// per-node assembly for one parameter (one workgroup per internal node P):
//   k_node_psi: X_ab = E_a^T S_b + S_a E_b,  PsiP = [[Psi_a, X_ab], [X_ab^T, Psi_b]],
//               gtr_P = <N_P, PsiP>
//   k_node_lam: dS_c = E_c + W_c^T,  Lam = N diag(dS_a, dS_b) N,
//               Vt_a = (N[a,b] W_b)^T,  Vt_b = (N[b,a] W_a)^T.
// ---------------------------------------------------------------------------
constexpr int AKMAX = 64;
__global__ void __launch_bounds__(256) k_node_psi(const double* Nn, const double* Sn, const double* E,
                                                  const double* Psi, double* PsiP, double* gtr, int kc, int heap0) {
  __shared__ double Xs[AKMAX * AKMAX];
  __shared__ double red[256];
  const int P = heap0 + blockIdx.x;
  const int a = 2 * P + 1, b = 2 * P + 2;
  const int m2 = 2 * kc;
  const long s2 = (long)kc * kc, ms = (long)m2 * m2;
  const double* N = Nn + P * ms;
  const double *Ea = E + a * s2, *Eb = E + b * s2, *Sa = Sn + a * s2, *Sb = Sn + b * s2;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < kc * kc; e += nt) {
    int i = e % kc, j = e / kc;
    double x = 0.0;
    for (int l = 0; l < kc; ++l)
      x += Ea[l + (long)i * kc] * Sb[l + (long)j * kc] + Sa[i + (long)l * kc] * Eb[l + (long)j * kc];
    Xs[e] = x;
  }
  __syncthreads();
  double* PP = PsiP + P * ms;
  double g = 0.0;
  for (int e = tid; e < m2 * m2; e += nt) {
    int i = e % m2, j = e / m2;
    double v;
    if (i < kc && j < kc) v = Psi[a * s2 + i + (long)j * kc];
    else if (i >= kc && j >= kc) v = Psi[b * s2 + (i - kc) + (long)(j - kc) * kc];
    else if (i < kc) v = Xs[i + (j - kc) * kc];
    else v = Xs[j + (i - kc) * kc];
    PP[e] = v;
    g += N[e] * v;
  }
  red[tid] = g;
  __syncthreads();
  for (int off = nt / 2; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  if (tid == 0) gtr[P] = red[0];
}

__global__ void __launch_bounds__(256) k_node_lam(const double* Nn, const double* E, const double* W, double* Lam,
                                                  double* Vt, double* scratch, int kc, int heap0) {
  __shared__ double dSa[AKMAX * AKMAX];
  __shared__ double dSb[AKMAX * AKMAX];
  const int P = heap0 + blockIdx.x;
  const int a = 2 * P + 1, b = 2 * P + 2;
  const int m2 = 2 * kc;
  const long s2 = (long)kc * kc, ms = (long)m2 * m2;
  const double* N = Nn + P * ms;
  const double *Ea = E + a * s2, *Eb = E + b * s2, *Wa = W + a * s2, *Wb = W + b * s2;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < kc * kc; e += nt) {
    int i = e % kc, j = e / kc;
    dSa[e] = Ea[e] + Wa[j + (long)i * kc];
    dSb[e] = Eb[e] + Wb[j + (long)i * kc];
  }
  __syncthreads();
  // T = N diag(dS_a, dS_b)
  double* T = scratch + (long)blockIdx.x * ms;
  for (int e = tid; e < m2 * m2; e += nt) {
    int i = e % m2, j = e / m2;
    double v = 0.0;
    if (j < kc) {
      for (int l = 0; l < kc; ++l) v += N[i + (long)l * m2] * dSa[l + j * kc];
    } else {
      for (int l = 0; l < kc; ++l) v += N[i + (long)(kc + l) * m2] * dSb[l + (j - kc) * kc];
    }
    T[e] = v;
  }
  __syncthreads();
  double* Lp = Lam + P * ms;
  for (int e = tid; e < m2 * m2; e += nt) {
    int i = e % m2, j = e / m2;
    double v = 0.0;
    for (int l = 0; l < m2; ++l) v += T[i + (long)l * m2] * N[l + (long)j * m2];
    Lp[e] = v;
  }
  // Vt_a(i,j) = sum_l W_b(l,i) N[b,a](l,j);  Vt_b(i,j) = sum_l W_a(l,i) N[a,b](l,j)
  for (int e = tid; e < kc * kc; e += nt) {
    int i = e % kc, j = e / kc;
    double va = 0.0, vb = 0.0;
    for (int l = 0; l < kc; ++l) {
      va += Wb[l + (long)i * kc] * N[(kc + l) + (long)j * m2];
      vb += Wa[l + (long)i * kc] * N[l + (long)(kc + j) * m2];
    }
    Vt[a * s2 + e] = va;
    Vt[b * s2 + e] = vb;
  }
}

// ---------------------------------------------------------------------------
// per-parameter work
// ---------------------------------------------------------------------------
hm_status param_prepare(FactorCtx& f, ParamBufs& pb, const double theta[4], const double* tF_prefix) {
  Model* m = f.m;
  const int n = m->n, kc = f.kc, levels = m->levels;
  const long pcnt = (long)n * levels * kc;
  const long s2 = (long)kc * kc;
  const double tau2 = theta[2], sigma2 = theta[3];
  if (pb.kind == 2) {  // K~_tau2 = I: no panels, identity leaves, Xi = G
    HM_CHECK(fill(m, pb.dF, pcnt, 0.0));
    HM_CHECK(leaf_affine(m, pb.dD, nullptr, 0.0, 1.0));
    HM_CHECK(lin2(m, pb.Xi, f.G, nullptr, pcnt, 1.0, 0.0));
  } else if (pb.kind == 3) {  // K~_sigma2 = (K~ - tau2 I)/sigma2: dF = F/(2 sigma2), Xi = (F - tau2 G)/sigma2
    HM_CHECK(lin2(m, pb.dF, f.F, nullptr, pcnt, 0.5 / sigma2, 0.0));
    HM_CHECK(leaf_affine(m, pb.dD, f.D, 1.0 / sigma2, -tau2 / sigma2));
    HM_CHECK(lin2(m, pb.Xi, f.F, f.G, pcnt, 1.0 / sigma2, -tau2 / sigma2));
  } else {  // Xi_c = B_cc G_c: leaves plus every sibling pair strictly inside c
    HM_CHECK(leaf_gemm(m, pb.dD, f.G, n, pb.Xi, n, levels * kc, 1.0, 0.0, 0, m->nleaves));
    if (levels >= 2) {
      const long ts = (long)kc * (levels - 1) * kc;
      ReduceJob rd{pb.dF, n, cs_block(kc), f.G, n, cs_prefix(kc), 2, levels, f.nU, ts, sel_all()};
      HM_CHECK(tree_reduce(m, rd));
      ExpandJob e1{pb.dF, n, cs_block(kc), pb.Xi, n, cs_prefix(kc), tF_prefix, ts, kc, 1, 0, 2, levels, 1.0, 1.0,
                   sel_all()};
      HM_CHECK(tree_expand(m, e1));
      ExpandJob e2{f.F, n, cs_block(kc), pb.Xi, n, cs_prefix(kc), f.nU, ts, kc, 1, 0, 2, levels, 1.0, 1.0,
                   sel_all()};
      HM_CHECK(tree_expand(m, e2));
    }
  }
  // leaf products Y = Dinv dD, Yt = dD Dinv
  const int nl = m->nl;
  const long ls = (long)nl * nl;
  HM_CHECK(gemm(m->stream, false, false, nl, nl, nl, 1.0, f.Dinv, nl, ls, pb.dD, nl, ls, 0.0, pb.Y, nl, ls,
                m->nleaves));
  HM_CHECK(gemm(m->stream, false, false, nl, nl, nl, 1.0, pb.dD, nl, ls, f.Dinv, nl, ls, 0.0, pb.Yt, nl, ls,
                m->nleaves));
  // E_c = dF_c^T G_c,  Psi_c = G_c^T Xi_c  (all non-root nodes)
  ReduceJob re{pb.dF, n, cs_block(kc), f.G, n, cs_block(kc), 1, levels, pb.E, s2, sel_all()};
  HM_CHECK(tree_reduce(m, re));
  ReduceJob rp{f.G, n, cs_block(kc), pb.Xi, n, cs_block(kc), 1, levels, pb.Psi, s2, sel_all()};
  HM_CHECK(tree_reduce(m, rp));
  return HM_OK;
}

// dG_c = K~_c^{-1} (dF_c - Xi_c) for every non-root node c, all depths at once:
//   K~_c^{-1} X = Dbar_c^{-1} X - sum_{P in subtree(c)} G_P N_P G_P^T X.
hm_status tangent_sweep(FactorCtx& f, ParamBufs& pb) {
  Model* m = f.m;
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
    for (int dP = 1; dP <= levels - 1; ++dP) HM_CHECK(node_apply_N(m, f.Nn, f.nT, ts, f.nU, us, kc, dP * kc, dP));
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

hm_status node_prep(FactorCtx& f) {
  Model* m = f.m;
  for (int d = 0; d < m->levels; ++d) {
    hipLaunchKernelGGL(k_node_prep, dim3(1 << d), dim3(256), 0, m->stream, f.Nn, f.Sn, f.Ncc, f.Nx, f.kc,
                       (1 << d) - 1);
    HM_LAUNCH_CHECK();
  }
  return HM_OK;
}

hm_status node_psi(FactorCtx& f, ParamBufs& pb, double* gtr) {
  Model* m = f.m;
  if (f.kc > AKMAX) {
    set_error("panel width exceeds 64");
    return HM_E_INVAL;
  }
  for (int d = 0; d < m->levels; ++d) {
    hipLaunchKernelGGL(k_node_psi, dim3(1 << d), dim3(256), 0, m->stream, f.Nn, f.Sn, pb.E, pb.Psi, pb.PsiP, gtr,
                       f.kc, (1 << d) - 1);
    HM_LAUNCH_CHECK();
  }
  return HM_OK;
}

hm_status node_lam(FactorCtx& f, ParamBufs& pb, double* scratch) {
  Model* m = f.m;
  for (int d = 0; d < m->levels; ++d) {
    hipLaunchKernelGGL(k_node_lam, dim3(1 << d), dim3(256), 0, m->stream, f.Nn, pb.E, pb.W, pb.Lam, pb.Vt, scratch,
                       f.kc, (1 << d) - 1);
    HM_LAUNCH_CHECK();
  }
  return HM_OK;
}

// Gh_c = dG_c N_P[c,c],  Hh_c = dG_c N_P[c,sib] S_sib
hm_status panel_products(FactorCtx& f, ParamBufs& pb) {
  Model* m = f.m;
  const int n = m->n, kc = f.kc, levels = m->levels;
  const long s2 = (long)kc * kc;
  ExpandJob e1{pb.dG, n, cs_block(kc), pb.Gh, n, cs_block(kc), f.Ncc, s2, kc, 0, 0, 1, levels, 1.0, 0.0, sel_all()};
  HM_CHECK(tree_expand(m, e1));
  ExpandJob e2{pb.dG, n, cs_block(kc), pb.Hh, n, cs_block(kc), f.Nx, s2, kc, 0, 0, 1, levels, 1.0, 0.0, sel_all()};
  HM_CHECK(tree_expand(m, e2));
  return HM_OK;
}

}  // namespace hm
