// Frozen compression of the oversampled sketches (used once, when the sketch
// state is created).
//
// Reading of Alg. 1 step 3 ("QR with column pivoting") with oversampling: each
// block is sampled with ell = r + p_os columns; its sample Y = Q R is
// Householder-factored, R's right singular vectors V (one-sided Jacobi, high
// relative accuracy for small singular values) keep
// k = min(r, #{sigma_i > tol sigma_1}) columns ordered by decreasing sigma (tol
// 1e-10 by default, or the caller's tolerance for ranks adapted per block),
// each signed so that its largest-magnitude entry is positive.  Column j of every
// block of a level is then scaled by one common factor d_j = exp(mean over the
// blocks keeping column j of log(sigma_1 / sigma_j)).  Omega V is the block's fixed
// test matrix (the sampling matrices are drawn once and kept fixed, Sec. 3.3), so
// Alg. 1 and Alg. 2 see a full-column-rank sample.  The blocks of a level share the
// columns of one patterned test matrix, so a scale common to all of them changes no
// block's sample beyond that scale: Q (diag R > 0), and so K~ and K~_j, are those of
// the unscaled directions, while R -- which Alg. 2 divides by -- is close to a
// multiple of an orthogonal matrix when the blocks' spectra are alike.
#include <cmath>

#include "hm_internal.h"

namespace hm {

constexpr int ELLMAX = 80;

__device__ double block_sum(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

// Householder QR of Y[a rows, 0:ell] for every block P at depth l-1 (left child
// a = 2P+1).  W: scratch copy, |a| x ell per block (ld |a|).  R: ell x ell per P.
__global__ void __launch_bounds__(256) k_house_qr(const double* Y, int ldy, double* W, double* R, int ell,
                                                  int l, int n) {
  __shared__ double red[256];
  const int pi = blockIdx.x;                 // block index at depth l-1
  const int m = n >> l;                      // rows of a left child at depth l
  const long r0 = (long)(2 * pi) * m;        // first row of a
  double* w = W + (long)pi * m * ell;
  double* Rp = R + (long)pi * ell * ell;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (long e = tid; e < (long)m * ell; e += nt) {
    int i = e % m, c = e / m;
    w[e] = Y[r0 + i + (long)c * ldy];
  }
  for (int e = tid; e < ell * ell; e += nt) Rp[e] = 0.0;
  __syncthreads();
  for (int j = 0; j < ell && j < m; ++j) {
    double* x = w + (long)j * m;
    double s = 0.0;
    for (int i = j + tid; i < m; i += nt) s += x[i] * x[i];
    s = block_sum(s, red);
    const double alpha = x[j];
    const double nx = sqrt(s);
    if (nx == 0.0) continue;  // zero column: R(j, .) stays zero in this column
    const double sg = (alpha >= 0.0) ? 1.0 : -1.0;
    const double v0 = alpha + sg * nx;
    const double vtv = s - alpha * alpha + v0 * v0;
    const double tau = 2.0 / vtv;
    __syncthreads();
    if (tid == 0) {
      x[j] = v0;  // v stored in place (rows j..m-1)
      Rp[j + j * ell] = -sg * nx;
    }
    __syncthreads();
    for (int c = j + 1; c < ell; ++c) {
      double* y = w + (long)c * m;
      double d = 0.0;
      for (int i = j + tid; i < m; i += nt) d += x[i] * y[i];
      d = block_sum(d, red);
      const double f = tau * d;
      for (int i = j + tid; i < m; i += nt) y[i] -= f * x[i];
      __syncthreads();
      if (tid == 0) Rp[j + c * ell] = y[j];
      __syncthreads();
    }
  }
}

// One-sided Jacobi SVD of R (ell x ell) per block; outputs V (ell x kc, zero
// padded), kept rank k, singular values.
__global__ void __launch_bounds__(256) k_jacobi_svd(const double* R, int ell, int rank, double tol, double* Vout,
                                                    int kc, int* kout, double* sout, int* flags) {
  __shared__ double A[ELLMAX * ELLMAX];
  __shared__ double V[ELLMAX * ELLMAX];
  __shared__ double sig[ELLMAX];
  __shared__ int order[ELLMAX];
  __shared__ int rotated;
  const int pi = blockIdx.x;
  const double* Rp = R + (long)pi * ell * ell;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < ell * ell; e += nt) {
    A[e] = Rp[e];
    V[e] = ((e % ell) == (e / ell)) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int mm = (ell + 1) & ~1;  // even number of players (one dummy if ell is odd)
  const int npair = mm / 2;
  const int G = 4;                // threads per pair
  int sweep = 0;
  for (; sweep < 60; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int st = 0; st < mm - 1; ++st) {
      const int pair = tid / G, lane = tid % G;
      int p = -1, q = -1;
      if (pair < npair) {
        int i0 = pair, i1 = mm - 1 - pair;
        auto pos = [&](int k) { return k == 0 ? 0 : ((k - 1 + st) % (mm - 1)) + 1; };
        p = pos(i0);
        q = pos(i1);
        if (p > q) { int t = p; p = q; q = t; }
      }
      double al = 0.0, be = 0.0, ga = 0.0;
      const bool act = (pair < npair) && q < ell;
      if (act)
        for (int i = lane; i < ell; i += G) {
          double ap = A[i + p * ell], aq = A[i + q * ell];
          al += ap * ap;
          be += aq * aq;
          ga += ap * aq;
        }
      // reduce within the group of G lanes (consecutive threads of one wavefront)
      for (int off = 1; off < G; off <<= 1) {
        al += __shfl_xor(al, off, G);
        be += __shfl_xor(be, off, G);
        ga += __shfl_xor(ga, off, G);
      }
      if (act && ga != 0.0 && fabs(ga) > 2.2e-16 * ell * sqrt(al * be)) {
        double zeta = (be - al) / (2.0 * ga);
        double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
        for (int i = lane; i < ell; i += G) {
          double ap = A[i + p * ell], aq = A[i + q * ell];
          A[i + p * ell] = c * ap - s * aq;
          A[i + q * ell] = s * ap + c * aq;
          double vp = V[i + p * ell], vq = V[i + q * ell];
          V[i + p * ell] = c * vp - s * vq;
          V[i + q * ell] = s * vp + c * vq;
        }
        if (lane == 0) rotated = 1;
      }
      __syncthreads();
    }
    if (!rotated) break;
    __syncthreads();
  }
  if (sweep == 60 && tid == 0) atomicOr(flags, (int)DF_JACOBI);
  for (int j = tid; j < ell; j += nt) {
    double s = 0.0;
    for (int i = 0; i < ell; ++i) s += A[i + j * ell] * A[i + j * ell];
    sig[j] = sqrt(s);
  }
  __syncthreads();
  if (tid == 0) {
    for (int j = 0; j < ell; ++j) order[j] = j;
    for (int a = 0; a < ell; ++a) {  // selection sort, decreasing sigma (stable on ties)
      int best = a;
      for (int b = a + 1; b < ell; ++b)
        if (sig[order[b]] > sig[order[best]]) best = b;
      int t = order[a]; order[a] = order[best]; order[best] = t;
    }
    const double s1 = sig[order[0]];
    int k = 0;
    if (s1 > 0.0)
      for (int j = 0; j < ell && k < rank; ++j)
        if (sig[order[j]] > tol * s1) ++k;
    kout[pi] = k;
    for (int j = 0; j < ell; ++j) sout[(long)pi * ell + j] = sig[order[j]];
  }
  __syncthreads();
  const int k = kout[pi];
  double* Vp = Vout + (long)pi * ell * kc;
  for (int j = tid; j < kc; j += nt) {
    if (j >= k) {
      for (int i = 0; i < ell; ++i) Vp[i + j * ell] = 0.0;
      continue;
    }
    const int src = order[j];
    int im = 0;
    double vm = -1.0;
    for (int i = 0; i < ell; ++i) {
      double a = fabs(V[i + src * ell]);
      if (a > vm) { vm = a; im = i; }
    }
    const double sg = (V[im + src * ell] < 0.0) ? -1.0 : 1.0;
    for (int i = 0; i < ell; ++i) Vp[i + j * ell] = sg * V[i + src * ell];
  }
}

// Common column scale of one level (see the header): V of nb blocks (ell x kc each,
// stride ell*kc), sorted singular values sig (ell per block), kept ranks k.
__global__ void __launch_bounds__(64) k_level_scale(double* V, const double* sig, const int* kk, int nb, int ell,
                                                    int kc) {
  __shared__ double d[ELLMAX];
  for (int j = threadIdx.x; j < kc; j += blockDim.x) {
    double acc = 0.0;
    int cnt = 0;
    for (int b = 0; b < nb; ++b)
      if (kk[b] > j) {
        acc += log(sig[(long)b * ell] / sig[(long)b * ell + j]);
        ++cnt;
      }
    d[j] = cnt ? exp(acc / cnt) : 1.0;
  }
  __syncthreads();
  for (long e = threadIdx.x; e < (long)nb * ell * kc; e += blockDim.x) {
    const int j = (int)((e / ell) % kc);
    V[e] *= d[j];
  }
}

hm_status sketch_compress(Model* m, const double* Y, int ldy, int ell, int l, int rank, double tol, double* W,
                          double* R, double* V, int kc, int* d_k, double* d_sig) {
  if (ell > ELLMAX) {
    set_error("rank + oversample exceeds 80");
    return HM_E_INVAL;
  }
  const int nb = 1 << (l - 1);
  hipLaunchKernelGGL(k_house_qr, dim3(nb), dim3(256), 0, m->stream, Y, ldy, W, R, ell, l, m->n);
  HM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_jacobi_svd, dim3(nb), dim3(256), 0, m->stream, R, ell, rank, tol, V, kc, d_k, d_sig,
                     m->d_flags);
  HM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_level_scale, dim3(1), dim3(64), 0, m->stream, V, d_sig, d_k, nb, ell, kc);
  HM_LAUNCH_CHECK();
  return HM_OK;
}

}  // namespace hm
