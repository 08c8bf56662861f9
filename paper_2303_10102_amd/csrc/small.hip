// Per-node small dense kernels (one workgroup per tree node, operands in LDS).
//
//  * k_chol_inv     Cholesky G = R^T R of a k x k Gram matrix (optionally shifted),
//                   with R and R^{-1}; the building block of the shifted Cholesky-QR
//                   used for Alg. 1 step 3 (QR with positive diagonal).
//  * k_alg2_fold    M = triu(W) + strict_tril(W)^T for Alg. 2 (W = Q^T dB R^{-1}):
//                   dQ = dB R^{-1} - Q M.
//  * k_node_lu      N_P = (J + S_P)^{-1} and log det(I + V^T U) for the Woodbury
//                   factor of node P (Sec. 3.1, App. C; Sylvester's identity), via
//                   the k x k Schur complement I - S_a S_b.
#include <cmath>

#include "hm_internal.h"

namespace hm {

constexpr int KMAX = 64;    // largest panel width handled in LDS

// ---------------------------------------------------------------------------
// Cholesky + triangular inverse of G (k x k, ld k), one node per workgroup.
// shift: if nonzero, G + s I with s = 11 (m k + k (k+1)) u ||.||_F^2, m = rows of
// the sketched block (shifted Cholesky-QR of Fukaya et al.); ||Y||_F^2 = tr(G).
// Zero columns (k_P < k) are kept as identity so padding stays exactly zero.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_chol_inv(const double* G, long gstride, double* R, double* Rinv,
                                                  long rstride, int k, const int* kblk, int heap0, int hstep,
                                                  int shift, long mrows, int* flags) {
  __shared__ double A[KMAX * KMAX];
  const int node = heap0 + blockIdx.x * hstep;
  // kept rank of the block whose left child is this node (kblk indexed by parent)
  const int kp = kblk ? kblk[(node - 1) >> 1] : k;
  const double* g = G + node * gstride;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < k * k; e += nt) {
    int i = e % k, j = e / k;
    double v = g[e];
    if (i >= kp || j >= kp) v = (i == j) ? 1.0 : 0.0;
    A[e] = v;
  }
  __syncthreads();
  if (shift) {
    __shared__ double tr;
    if (tid == 0) {
      double t = 0.0;
      for (int i = 0; i < kp; ++i) t += A[i + i * k];
      tr = 11.0 * ((double)mrows * kp + (double)kp * (kp + 1)) * 1.1102230246251565e-16 * t;
    }
    __syncthreads();
    for (int i = tid; i < kp; i += nt) A[i + i * k] += tr;
    __syncthreads();
  }
  // right-looking Cholesky, lower factor in A (column-major)
  __shared__ int bad;
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    if (tid == 0) {
      double d = A[j + j * k];
      if (!(d > 0.0)) { bad = 1; d = 1.0; }
      A[j + j * k] = sqrt(d);
    }
    __syncthreads();
    const double piv = A[j + j * k];
    for (int i = j + 1 + tid; i < k; i += nt) A[i + j * k] /= piv;
    __syncthreads();
    const int r = k - j - 1;
    for (int e = tid; e < r * r; e += nt) {
      int i = j + 1 + e % r, l = j + 1 + e / r;
      if (i >= l) A[i + l * k] -= A[i + j * k] * A[l + j * k];
    }
    __syncthreads();
  }
  if (bad && tid == 0) atomicOr(flags, (int)DF_QR_FAIL);
  // R = L^T (upper), Rinv = (L^{-1})^T; column c of L^{-1} by forward substitution in LDS
  __shared__ double X[KMAX * KMAX];   // X[c + i*k] = (L^{-1})(i, c)
  double* Ro = R + node * rstride;
  double* Ri = Rinv + node * rstride;
  for (int e = tid; e < k * k; e += nt) {
    int i = e % k, j = e / k;
    Ro[e] = (i <= j) ? A[j + i * k] : 0.0;  // R(i,j) = L(j,i)
  }
  for (int c = tid; c < k; c += nt) {
    for (int i = 0; i < c; ++i) X[c + i * k] = 0.0;
    for (int i = c; i < k; ++i) {
      // four independent partial sums break the FMA dependency chain
      double s0 = (i == c) ? 1.0 : 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      int l = c;
      for (; l + 3 < i; l += 4) {
        s0 -= A[i + l * k] * X[c + l * k];
        s1 -= A[i + (l + 1) * k] * X[c + (l + 1) * k];
        s2 -= A[i + (l + 2) * k] * X[c + (l + 2) * k];
        s3 -= A[i + (l + 3) * k] * X[c + (l + 3) * k];
      }
      for (; l < i; ++l) s0 -= A[i + l * k] * X[c + l * k];
      X[c + i * k] = ((s0 + s1) + (s2 + s3)) / A[i + i * k];
    }
  }
  __syncthreads();
  for (int e = tid; e < k * k; e += nt) Ri[e] = X[e];   // Rinv(c, i) = (L^{-1})(i, c)
}

// M = triu(W) + strict_tril(W)^T, W k x k (ld k) per node; zero outside k_P.
__global__ void k_alg2_fold(const double* W, double* M, long stride, int k, int heap0) {
  const int node = heap0 + blockIdx.x;
  const double* w = W + node * stride;
  double* mm = M + node * stride;
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
    int i = e % k, j = e / k;
    mm[e] = (i <= j) ? w[i + j * k] + ((i < j) ? w[j + i * k] : 0.0) : 0.0;
  }
}

// ---------------------------------------------------------------------------
// Node factor.  M_P = I + J S_P = [[I, S_b], [S_a, I]] with S_c = F_c^T G_c.  With
// the Schur complement Sig = I - S_a S_b (for SPD K~_P its eigenvalues lie in
// (0, 1]):  det M_P = det Sig  and
//   M_P^{-1} = [[I + S_b Sig^{-1} S_a, -S_b Sig^{-1}], [-Sig^{-1} S_a, Sig^{-1}]],
//   N_P = M_P^{-1} J = [[-S_b Sig^{-1}, I + S_b Sig^{-1} S_a], [Sig^{-1}, -Sig^{-1} S_a]] = (J + S_P)^{-1}.
// logdet_P = log det M_P (> 0 required, else the node is flagged not SPD).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_node_lu(const double* S, long sstride, double* Nout, long nstride,
                                                 double* logdet, int k, int heap0, int* flags) {
  __shared__ double Sa[KMAX * KMAX];
  __shared__ double Sb[KMAX * KMAX];
  __shared__ double A[KMAX * KMAX];     // Sig, then its LU factors
  __shared__ double Si[KMAX * KMAX];    // Sig^{-1}
  __shared__ int piv[KMAX];
  __shared__ double sgn, lsum;
  const int P = heap0 + blockIdx.x;
  const int a = 2 * P + 1, b = 2 * P + 2;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int kk = k * k;
  for (int e = tid; e < kk; e += nt) {
    Sa[e] = S[a * sstride + e];
    Sb[e] = S[b * sstride + e];
  }
  __syncthreads();
  for (int e = tid; e < kk; e += nt) {
    int i = e % k, j = e / k;
    double v = (i == j) ? 1.0 : 0.0;
    for (int l = 0; l < k; ++l) v -= Sa[i + l * k] * Sb[l + j * k];
    A[e] = v;
  }
  if (tid == 0) { sgn = 1.0; lsum = 0.0; }
  __syncthreads();
  // LU with partial pivoting; the pivot search is done by the first wavefront
  for (int j = 0; j < k; ++j) {
    if (tid < 64) {
      double best = -1.0;
      int bi = j;
      for (int i = j + tid; i < k; i += 64) {
        double v = fabs(A[i + j * k]);
        if (v > best) { best = v; bi = i; }
      }
      for (int off = 32; off > 0; off >>= 1) {
        double ob = __shfl_xor(best, off, 64);
        int oi = __shfl_xor(bi, off, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (tid == 0) piv[j] = bi;
    }
    __syncthreads();
    const int pr = piv[j];
    if (pr != j)
      for (int c = tid; c < k; c += nt) {
        double t = A[j + c * k];
        A[j + c * k] = A[pr + c * k];
        A[pr + c * k] = t;
      }
    __syncthreads();
    const double d = A[j + j * k];
    if (tid == 0) {
      if (pr != j) sgn = -sgn;
      if (d < 0.0) sgn = -sgn;
      lsum += log(fabs(d));
    }
    if (d != 0.0)
      for (int i = j + 1 + tid; i < k; i += nt) A[i + j * k] /= d;
    __syncthreads();
    const int r = k - j - 1;
    for (int e = tid; e < r * r; e += nt) {
      int i = j + 1 + e % r, c = j + 1 + e / r;
      A[i + c * k] -= A[i + j * k] * A[j + c * k];
    }
    __syncthreads();
  }
  if (tid == 0) {
    logdet[P] = lsum;
    if (!(sgn > 0.0) || !isfinite(lsum)) atomicOr(flags, (int)DF_NOT_SPD_NODE);
  }
  // Sig^{-1}: column c solves L U x = P e_c
  for (int c = tid; c < k; c += nt) {
    double* x = Si + c * k;
    for (int i = 0; i < k; ++i) x[i] = (i == c) ? 1.0 : 0.0;
    for (int i = 0; i < k; ++i) {
      int q = piv[i];
      if (q != i) { double t = x[i]; x[i] = x[q]; x[q] = t; }
    }
    for (int i = 0; i < k; ++i) {
      double s0 = x[i], s1 = 0.0, s2 = 0.0, s3 = 0.0;
      int l = 0;
      for (; l + 3 < i; l += 4) {
        s0 -= A[i + l * k] * x[l];
        s1 -= A[i + (l + 1) * k] * x[l + 1];
        s2 -= A[i + (l + 2) * k] * x[l + 2];
        s3 -= A[i + (l + 3) * k] * x[l + 3];
      }
      for (; l < i; ++l) s0 -= A[i + l * k] * x[l];
      x[i] = (s0 + s1) + (s2 + s3);
    }
    for (int i = k - 1; i >= 0; --i) {
      double s0 = x[i], s1 = 0.0, s2 = 0.0, s3 = 0.0;
      int l = i + 1;
      for (; l + 3 < k; l += 4) {
        s0 -= A[i + l * k] * x[l];
        s1 -= A[i + (l + 1) * k] * x[l + 1];
        s2 -= A[i + (l + 2) * k] * x[l + 2];
        s3 -= A[i + (l + 3) * k] * x[l + 3];
      }
      for (; l < k; ++l) s0 -= A[i + l * k] * x[l];
      x[i] = ((s0 + s1) + (s2 + s3)) / A[i + i * k];
    }
  }
  __syncthreads();
  // P1 = S_b Sig^{-1} -> A (LU no longer needed)
  for (int e = tid; e < kk; e += nt) {
    int i = e % k, j = e / k;
    double v = 0.0;
    for (int l = 0; l < k; ++l) v += Sb[i + l * k] * Si[l + j * k];
    A[e] = v;
  }
  __syncthreads();
  const int m = 2 * k;
  double* No = Nout + P * nstride;
  for (int e = tid; e < kk; e += nt) {
    int i = e % k, j = e / k;
    double n12 = (i == j) ? 1.0 : 0.0, n22 = 0.0;
    for (int l = 0; l < k; ++l) {
      n12 += A[i + l * k] * Sa[l + j * k];
      n22 -= Si[i + l * k] * Sa[l + j * k];
    }
    No[i + (long)j * m] = -A[e];                 // N11 = -S_b Sig^{-1}
    No[i + (long)(k + j) * m] = n12;             // N12 = I + S_b Sig^{-1} S_a
    No[(k + i) + (long)j * m] = Si[e];           // N21 = Sig^{-1}
    No[(k + i) + (long)(k + j) * m] = n22;       // N22 = -Sig^{-1} S_a
  }
}

hm_status chol_inv_nodes(Model* m, const double* G, long gstride, double* R, double* Rinv, long rstride,
                         int k, const int* d_kblk, int heap0, int hstep, int cnt, int shift, long mrows) {
  if (k > KMAX) {
    set_error("panel width exceeds the per-node LDS limit (64)");
    return HM_E_INVAL;
  }
  hipLaunchKernelGGL(k_chol_inv, dim3(cnt), dim3(256), 0, m->stream, G, gstride, R, Rinv, rstride, k, d_kblk,
                     heap0, hstep, shift, mrows, m->d_flags);
  HM_LAUNCH_CHECK();
  return HM_OK;
}

hm_status alg2_fold_nodes(Model* m, const double* W, double* M, long stride, int k, int heap0, int cnt) {
  hipLaunchKernelGGL(k_alg2_fold, dim3(cnt), dim3(256), 0, m->stream, W, M, stride, k, heap0);
  HM_LAUNCH_CHECK();
  return HM_OK;
}

hm_status node_lu(Model* m, const double* S, long sstride, double* Nout, long nstride, double* logdet, int k,
                  int heap0, int cnt) {
  if (k > KMAX) {
    set_error("panel width exceeds the per-node LDS limit (64)");
    return HM_E_INVAL;
  }
  hipLaunchKernelGGL(k_node_lu, dim3(cnt), dim3(256), 0, m->stream, S, sstride, Nout, nstride, logdet, k, heap0,
                     m->d_flags);
  HM_LAUNCH_CHECK();
  return HM_OK;
}

}  // namespace hm
