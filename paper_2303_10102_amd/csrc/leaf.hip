// Leaf blocks: extraction from the stacked-identity sample, Cholesky, log-det,
// explicit inverses.
//
// The leaf blocks of K~ are read from (K - sum_l H_l) [I; I; ...] (Sec. 3.2,
// eq. "leaf sample") and symmetrised.  The factorisation K~ = Dbar * prod(I + U V^T)
// starts by factoring out the block-diagonal Dbar of leaf blocks (App. C, eq.
// "factor out leaf"); its log-determinant is 2 sum log diag(chol(D_L)).
#include <cmath>
#include <vector>

#include "hm_build.h"
#include "hm_internal.h"

namespace hm {

// D_L = (Z_L + Z_L^T)/2 with Z rows in tree order (ld ldz), leaf-major output.
// 32 x 32 tiles: the tile and its mirror are staged through LDS so both reads and
// the write are coalesced.
__global__ void __launch_bounds__(256) k_leaf_sym(const double* Z, int ldz, double* D, int nl, double scale) {
  __shared__ double t0[32][33], t1[32][33];
  const int L = blockIdx.z;
  const long r0 = (long)L * nl;
  const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  for (int q = ty; q < 32; q += 8) {
    const int i = i0 + tx, j = j0 + q;        // element (i, j) of the tile
    t0[q][tx] = (i < nl && j < nl) ? Z[r0 + i + (long)j * ldz] : 0.0;
    const int i2 = j0 + tx, j2 = i0 + q;      // element (j0 + tx, i0 + q) of the mirror tile
    t1[q][tx] = (i2 < nl && j2 < nl) ? Z[r0 + i2 + (long)j2 * ldz] : 0.0;
  }
  __syncthreads();
  double* Dl = D + (long)L * nl * nl;
  for (int q = ty; q < 32; q += 8) {
    const int i = i0 + tx, j = j0 + q;
    // Z(j, i) = mirror tile element (row j - j0 = q, column i - i0 = tx) = t1[tx][q]
    if (i < nl && j < nl) Dl[i + (long)j * nl] = 0.5 * scale * (t0[q][tx] + t1[tx][q]);
  }
}

hm_status leaf_sym(Model* m, const double* Z, int ldz, double* D) {
  const int nl = m->nl;
  hipLaunchKernelGGL(k_leaf_sym, dim3(ceil_div(nl, 32), ceil_div(nl, 32), m->nleaves), dim3(256), 0, m->stream, Z,
                     ldz, D, nl, 1.0);
  HM_LAUNCH_CHECK();
  return HM_OK;
}

// Block widths of the leaf Cholesky and the largest leaf each handles: the panel of
// the block column (all rows below the diagonal block, CB + 1 doubles per row) is
// held in LDS, 135 KB at width 32 and 512 rows, 153 KB at width 16 and 1152 rows.
constexpr int CNB = 32;
constexpr int NLMAX = 512;
constexpr int CNB_WIDE = 16;
constexpr int NLMAX_WIDE = 1152;

// Right-looking blocked Cholesky of every leaf, one block column per launch:
// k_chol_panel factors the diagonal block and solves the rows below it (the
// panel is held in LDS); the trailing update A22 -= L21 L21^T is a batched
// MFMA GEMM over all leaves.  logdet[L] accumulates 2 sum log L_ii; a
// non-positive pivot sets a flag and is replaced by 1 so the kernel completes.
template <int CNB, int NLMAX>
__global__ void __launch_bounds__(256) k_chol_panel(double* W, int nl, int jb, double* logdet, int* flags) {
  __shared__ double panel[NLMAX * (CNB + 1)];   // rows jb..nl-1 of the block column
  const int L = blockIdx.x;
  double* A = W + (long)L * nl * nl;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int nb = min(CNB, nl - jb);
  const int rows = nl - jb;
  constexpr int LD = CNB + 1;
  for (int e = tid; e < rows * nb; e += nt) {
    int i = e % rows, t = e / rows;
    panel[i * LD + t] = A[(jb + i) + (long)(jb + t) * nl];
  }
  __syncthreads();
  double lsum = 0.0;
  int bad = 0;
  for (int t = 0; t < nb; ++t) {
    if (tid == 0) {
      double d = panel[t * LD + t];
      if (!(d > 0.0)) { bad = 1; d = 1.0; }
      d = sqrt(d);
      panel[t * LD + t] = d;
      lsum += 2.0 * log(d);
    }
    __syncthreads();
    const double piv = panel[t * LD + t];
    for (int i = t + 1 + tid; i < rows; i += nt) panel[i * LD + t] /= piv;
    __syncthreads();
    const int rr = rows - t - 1, cc = nb - t - 1;
    for (int e = tid; e < rr * cc; e += nt) {
      int i = t + 1 + e % rr, u = t + 1 + e / rr;
      if (i >= u) panel[i * LD + u] -= panel[i * LD + t] * panel[u * LD + t];
    }
    __syncthreads();
  }
  for (int e = tid; e < rows * nb; e += nt) {
    int i = e % rows, t = e / rows;
    A[(jb + i) + (long)(jb + t) * nl] = (i >= t) ? panel[i * LD + t] : 0.0;
  }
  if (tid == 0) {
    logdet[L] = (jb == 0 ? 0.0 : logdet[L]) + lsum;
    if (bad) atomicOr(flags, (int)DF_NOT_SPD_LEAF);
  }
}

// The same step for leaves of at most 256 rows, with the panel in registers: thread i
// holds row jb + i of the block column.  Step t broadcasts column t of the diagonal
// block (rows < nb) through LDS, one barrier per step; every row then scales its
// entry t by the pivot and updates its entries right of t with one multiply-add each.
template <int CB>
__global__ void __launch_bounds__(256) k_chol_panel_r(double* W, int nl, int jb, double* logdet, int* flags) {
  __shared__ double colt[2][CB];
  __shared__ double red[4];
  const int L = blockIdx.x;
  double* A = W + (long)L * nl * nl;
  const int i = threadIdx.x;
  const int nb = min(CB, nl - jb), rows = nl - jb;
  const bool act = i < rows;
  double R[CB];
#pragma unroll
  for (int t = 0; t < CB; ++t) R[t] = (act && t < nb) ? A[(jb + i) + (long)(jb + t) * nl] : 0.0;
  double myl = 0.0;   // 2 log of this row's pivot (rows < nb)
  bool bad = false;
#pragma unroll
  for (int t = 0; t < CB; ++t) {
    if (t < nb) {
      double* cb = colt[t & 1];
      if (i < nb) cb[i] = R[t];
      __syncthreads();
      double d = cb[t];
      if (!(d > 0.0)) {
        bad = true;
        d = 1.0;
      }
      const double piv = sqrt(d), rp = 1.0 / piv;
      if (i == t) {
        R[t] = piv;
        myl = 2.0 * log(piv);
      } else if (i > t) {
        R[t] = R[t] / piv;
      }
      const double lt = R[t];
      // Every row updates every entry right of t: an entry above the diagonal (u > i)
      // or past the panel (u >= nb, stale broadcast) never feeds an entry on or below
      // the diagonal and is never written out.  The broadcast reads are all issued
      // before the first multiply-add (the empty asm takes each value).
      double c_[CB];
#pragma unroll
      for (int u = t + 1; u < CB; ++u) c_[u] = cb[u];
#pragma unroll
      for (int u = t + 1; u < CB; ++u) asm volatile("" : "+v"(c_[u]));
#pragma unroll
      for (int u = t + 1; u < CB; ++u) R[u] -= lt * (c_[u] * rp);
#pragma unroll
      for (int u = t + 1; u < CB; ++u) asm volatile("" : "+v"(R[u]));
    }
  }
  if (act) {
#pragma unroll
    for (int t = 0; t < CB; ++t)
      if (t < nb) A[(jb + i) + (long)(jb + t) * nl] = (i >= t) ? R[t] : 0.0;
  }
  // log det contribution: the pivots' logs, summed over the block
  double ls = (i < nb) ? myl : 0.0;
  for (int off = 32; off > 0; off >>= 1) ls += __shfl_xor(ls, off, 64);
  if ((i & 63) == 0) red[i >> 6] = ls;
  __syncthreads();
  if (i == 0) {
    logdet[L] = (jb == 0 ? 0.0 : logdet[L]) + ((red[0] + red[1]) + (red[2] + red[3]));
    if (bad) atomicOr(flags, (int)DF_NOT_SPD_LEAF);
  }
}

// Inverse of each CNB x CNB diagonal block of the lower factor, written into the
// same position of Linv.  One workgroup per (block, leaf); thread c < nb solves
// column c by forward substitution with the block in LDS.
template <int CNB>
__global__ void __launch_bounds__(64) k_tri_inv_diag(const double* Lf, double* Linv, int nl) {
  __shared__ double B[CNB * (CNB + 1)];
  __shared__ double X[CNB * (CNB + 1)];
  const int k = blockIdx.x, L = blockIdx.y;
  const int o = k * CNB;
  const int nb = min(CNB, nl - o);
  const double* A = Lf + (long)L * nl * nl + o + (long)o * nl;
  double* Y = Linv + (long)L * nl * nl + o + (long)o * nl;
  constexpr int LD = CNB + 1;
  for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
    int i = e % nb, j = e / nb;
    B[i + j * LD] = A[i + (long)j * nl];
  }
  __syncthreads();
  const int c = threadIdx.x;
  if (c < nb) {
    for (int i = 0; i < nb; ++i) {
      double v = (i == c) ? 1.0 : 0.0;
      for (int q = c; q < i; ++q) v -= B[i + q * LD] * X[q + c * LD];
      X[i + c * LD] = (i < c) ? 0.0 : v / B[i + i * LD];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
    int i = e % nb, j = e / nb;
    Y[i + (long)j * nl] = X[i + j * LD];
  }
}

// Dinv_L = L^{-T} L^{-1};  logdet_leaf[L] = log det D_L.  work: nleaves*nl*nl doubles.
// The inverse of the lower factor is assembled bottom-up from the diagonal-block
// inverses: for adjacent groups g0 (rows o..o+s0) and g1 (o+s0..o+s0+s1),
//   inv([[A, 0], [B, C]]) = [[A^-1, 0], [-C^-1 B A^-1, C^-1]]   (two batched GEMMs per merge).
hm_status leaf_factor(Model* m, const double* D, double* Dinv, double* logdet_leaf, double* work) {
  const int nl = m->nl;
  if (nl > NLMAX_WIDE) {
    set_error("leaf size exceeds 1152");
    return HM_E_INVAL;
  }
  const bool wide = nl > NLMAX;              // long panels: narrower block columns
  const int cb = wide ? CNB_WIDE : CNB;
  const long ls = (long)nl * nl;
  const long sz = (long)m->nleaves * ls;
  const int nlv = m->nleaves;
  HM_HIP(hipMemcpyAsync(work, D, sz * sizeof(double), hipMemcpyDeviceToDevice, m->stream));
  for (int jb = 0; jb < nl; jb += cb) {
    if (wide)
      hipLaunchKernelGGL((k_chol_panel<CNB_WIDE, NLMAX_WIDE>), dim3(nlv), dim3(256), 0, m->stream, work, nl, jb,
                         logdet_leaf, m->d_flags);
    else if (nl <= 256)
      hipLaunchKernelGGL((k_chol_panel_r<CNB>), dim3(nlv), dim3(256), 0, m->stream, work, nl, jb, logdet_leaf,
                         m->d_flags);
    else
      hipLaunchKernelGGL((k_chol_panel<CNB, NLMAX>), dim3(nlv), dim3(256), 0, m->stream, work, nl, jb,
                         logdet_leaf, m->d_flags);
    HM_LAUNCH_CHECK();
    const int j2 = jb + cb;
    if (j2 < nl) {
      const int r2 = nl - j2;
      const double* L21 = work + j2 + (long)jb * nl;
      HM_CHECK(gemm(m->stream, false, true, r2, r2, cb, -1.0, L21, nl, ls, L21, nl, ls, 1.0,
                    work + j2 + (long)j2 * nl, nl, ls, nlv));
    }
  }
  // Linv (lower) in Dinv
  HM_CHECK(fill(m, Dinv, sz, 0.0));
  const int nblk = ceil_div(nl, cb);
  if (wide)
    hipLaunchKernelGGL(k_tri_inv_diag<CNB_WIDE>, dim3(nblk, nlv), dim3(64), 0, m->stream, work, Dinv, nl);
  else
    hipLaunchKernelGGL(k_tri_inv_diag<CNB>, dim3(nblk, nlv), dim3(64), 0, m->stream, work, Dinv, nl);
  HM_LAUNCH_CHECK();
  // groups: [start, size); merge neighbours pairwise until one group spans the leaf
  std::vector<int> gs, gz;
  for (int k = 0; k < nblk; ++k) {
    gs.push_back(k * cb);
    gz.push_back(std::min(cb, nl - k * cb));
  }
  double* T = m->d_ws;   // scratch for B A^{-1}: needs nleaves * s1 * s0 <= nleaves * nl^2 / 4
  const long tneed = (long)nlv * (nl / 2 + cb) * (nl / 2 + cb);
  if (tneed > 3L * m->n * m->cmax) {
    set_error("leaf_factor: scratch too small");
    return HM_E_INVAL;
  }
  while (gs.size() > 1) {
    std::vector<int> ns, nz;
    for (size_t g = 0; g + 1 < gs.size(); g += 2) {
      const int o = gs[g], s0 = gz[g], s1 = gz[g + 1];
      const long tst = (long)s1 * s0;
      // T = B A^{-1}:  B = L[o+s0 : o+s0+s1, o : o+s0],  A^{-1} = Linv[o : o+s0, o : o+s0]
      HM_CHECK(gemm(m->stream, false, false, s1, s0, s0, 1.0, work + (o + s0) + (long)o * nl, nl, ls,
                    Dinv + o + (long)o * nl, nl, ls, 0.0, T, s1, tst, nlv));
      // Linv[o+s0 :, o : o+s0] = -C^{-1} T
      HM_CHECK(gemm(m->stream, false, false, s1, s0, s1, -1.0, Dinv + (o + s0) + (long)(o + s0) * nl, nl, ls, T,
                    s1, tst, 0.0, Dinv + (o + s0) + (long)o * nl, nl, ls, nlv));
      ns.push_back(o);
      nz.push_back(s0 + s1);
    }
    if (gs.size() % 2) {
      ns.push_back(gs.back());
      nz.push_back(gz.back());
    }
    gs.swap(ns);
    gz.swap(nz);
  }
  // Dinv = Linv^T Linv (into work, then back)
  HM_CHECK(gemm(m->stream, true, false, nl, nl, nl, 1.0, Dinv, nl, ls, Dinv, nl, ls, 0.0, work, nl, ls, nlv));
  HM_HIP(hipMemcpyAsync(Dinv, work, sz * sizeof(double), hipMemcpyDeviceToDevice, m->stream));
  return HM_OK;
}

}  // namespace hm
