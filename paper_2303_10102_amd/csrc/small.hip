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

// dst[c * ds] -= f * src[c * ss] for c = c0, c0 + step, ... < c1, four updates at a time
// with every read issued before the writes (callers guarantee dst and src never overlap),
// so the LDS round trips of one group overlap.
__device__ __forceinline__ void axpy_strided(double* dst, long ds, const double* src, long ss, double f, int c0,
                                             int c1, int step) {
  int c = c0;
  for (; c + 3 * step < c1; c += 4 * step) {
    const double s0 = src[c * ss], s1 = src[(c + step) * ss], s2 = src[(c + 2 * step) * ss],
                 s3 = src[(c + 3 * step) * ss];
    const double d0 = dst[c * ds], d1 = dst[(c + step) * ds], d2 = dst[(c + 2 * step) * ds],
                 d3 = dst[(c + 3 * step) * ds];
    dst[c * ds] = d0 - f * s0;
    dst[(c + step) * ds] = d1 - f * s1;
    dst[(c + 2 * step) * ds] = d2 - f * s2;
    dst[(c + 3 * step) * ds] = d3 - f * s3;
  }
  for (; c < c1; c += step) dst[c * ds] -= f * src[c * ss];
}

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
  // Right-looking Cholesky fused with the forward elimination of L Y = I, one barrier
  // per column.  Step j reads column j of the Schur-updated A (final after step j-1)
  // and row j of Y, and writes only columns / rows past j, so nothing it reads is
  // written in the same step.  With d_j = A(j, j), l_ij = A(i, j) / sqrt(d_j):
  //   A(i, l) -= A(i, j) A(l, j) / d_j          (j < l <= i)
  //   Y(i, c) -= A(i, j) / d_j * Y(j, c)        (i > j, c <= j)
  // and L^{-1}(i, c) = Y(i, c) / sqrt(d_i).  A pivot that is not positive is flagged
  // and taken as 1.
  __shared__ double Y[KMAX * KMAX];
  for (int e = tid; e < k * k; e += nt) Y[e] = (e % k == e / k) ? 1.0 : 0.0;
  __syncthreads();
  // Lane i of every wavefront owns row i (k <= 64); wavefront w takes the columns
  // congruent to w modulo the wavefront count, so the pivot-row operand is a broadcast.
  bool bad = false;
  const int lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
  for (int j = 0; j < k; ++j) {
    double d = A[j + j * k];
    if (!(d > 0.0)) { bad = true; d = 1.0; }
    const double rd = 1.0 / d;
    const int i = lane;
    if (i > j && i < k) {
      const double f = A[i + j * k] * rd;
      axpy_strided(A + i, k, A + (long)j * k, 1, f, j + 1 + wave, i + 1, nw);   // column j is not written
      axpy_strided(Y + i, k, Y + j, k, f, wave, j + 1, nw);                     // row j is not written
    }
    __syncthreads();
  }
  if (bad && tid == 0) atomicOr(flags, (int)DF_QR_FAIL);
  // R = L^T (upper), Rinv = (L^{-1})^T
  double* Ro = R + node * rstride;
  double* Ri = Rinv + node * rstride;
  for (int e = tid; e < k * k; e += nt) {
    const int i = e % k, j = e / k;
    double dj = A[j + j * k], di = A[i + i * k];
    if (!(dj > 0.0)) dj = 1.0;
    if (!(di > 0.0)) di = 1.0;
    // R(i, j) = L(j, i) for i <= j
    Ro[e] = (i < j) ? A[j + i * k] / sqrt(di) : (i == j ? sqrt(di) : 0.0);
    // Rinv(i, j) = L^{-1}(j, i) = Y(j, i) / sqrt(d_j) for j >= i
    Ri[e] = (j >= i) ? Y[j + i * k] / sqrt(dj) : 0.0;
  }
}

// M = triu(W) + strict_tril(W)^T, W k x k (ld k) per node; zero outside k_P.  trans:
// the node holds W^T instead of W.
__global__ void k_alg2_fold(const double* W, double* M, long stride, int k, int heap0, int trans) {
  const int node = heap0 + blockIdx.x;
  const double* w = W + node * stride;
  double* mm = M + node * stride;
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
    const int i = e % k, j = e / k;
    const double wij = trans ? w[j + i * k] : w[i + j * k];
    const double wji = trans ? w[i + j * k] : w[j + i * k];
    mm[e] = (i <= j) ? wij + ((i < j) ? wji : 0.0) : 0.0;
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
  __shared__ double A[KMAX * KMAX];     // Sig, eliminated in place
  __shared__ double Si[KMAX * KMAX];    // the accumulated row operations, then Sig^{-1}
  __shared__ int piv[KMAX];
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
  for (int e = tid; e < kk; e += nt) Si[e] = (e % k == e / k) ? 1.0 : 0.0;
  __syncthreads();
  // Gauss-Jordan elimination with partial pivoting on [Sig | I], one barrier per
  // column.  Every wavefront finds the pivot of column j itself (the largest |A(i, j)|
  // over rows not yet used, ties to the lower row; lane i holds row i), so no barrier
  // separates the search from the update; the pivot row p is only read in step j.
  // All other rows are eliminated: A(i, c) -= A(i, j) / A(p, j) A(p, c) for c > j and
  // the same on Y = Si, after which Sig^{-1}(j, :) = Y(p_j, :) / A(p_j, j) and
  // det Sig = sign(pivot permutation) * prod_j A(p_j, j).
  const int lane = tid & 63;
  bool used = lane >= k;
  __shared__ double pval[KMAX];
  for (int j = 0; j < k; ++j) {
    double best = -1.0;
    int bi = KMAX;
    if (!used) {
      best = fabs(A[lane + j * k]);
      if (!(best <= INFINITY)) best = INFINITY;   // NaN ranks first: the order stays total
      bi = lane;
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    const int p = bi;
    if (lane == p) used = true;
    const double pv = A[p + j * k];
    if (tid == 0) { piv[j] = p; pval[j] = pv; }
    const double rp = (pv != 0.0) ? 1.0 / pv : 0.0;
    // lane i owns row i; wavefront w takes columns congruent to w (pivot row: broadcast)
    if (lane < k && lane != p) {
      const double f = A[lane + j * k] * rp;
      const int wave = tid >> 6, nw = nt >> 6;
      axpy_strided(A + lane, k, A + p, k, f, j + 1 + wave, k, nw);   // row p is not written
      axpy_strided(Si + lane, k, Si + p, k, f, wave, k, nw);
    }
    __syncthreads();
  }
  // Sig^{-1}(j, c) = Y(p_j, c) / A(p_j, j), into A (column j of A is read no more)
  for (int e = tid; e < kk; e += nt) {
    const int j = e % k, c = e / k;
    A[e] = Si[piv[j] + c * k] / pval[j];
  }
  __syncthreads();
  for (int e = tid; e < kk; e += nt) Si[e] = A[e];
  if (tid == 0) {
    // log |det| and the sign: pivot signs times the parity of the pivot permutation
    double ls = 0.0;
    int neg = 0;
    for (int j = 0; j < k; ++j) {
      ls += log(fabs(pval[j]));
      if (pval[j] < 0.0) ++neg;
    }
    unsigned long long seen = 0ull;   // k <= 64
    int cycles = 0;
    for (int j = 0; j < k; ++j) {
      if ((seen >> j) & 1ull) continue;
      ++cycles;
      for (int q = j; !((seen >> q) & 1ull); q = piv[q]) seen |= 1ull << q;
    }
    const bool positive = (((k - cycles) + neg) % 2) == 0;
    logdet[P] = ls;
    if (!positive || !isfinite(ls)) atomicOr(flags, (int)DF_NOT_SPD_NODE);
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

hm_status alg2_fold_nodes(Model* m, const double* W, double* M, long stride, int k, int heap0, int cnt, bool trans) {
  hipLaunchKernelGGL(k_alg2_fold, dim3(cnt), dim3(256), 0, m->stream, W, M, stride, k, heap0, trans ? 1 : 0);
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
