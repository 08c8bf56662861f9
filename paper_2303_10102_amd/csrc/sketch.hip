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

// R factors of the level's samples by a tall-skinny Householder QR: each block's rows are
// cut into chunks of CH, every chunk is factored in LDS by one workgroup, the chunks' R
// factors are stacked and factored again, until one R per block remains (the same R up
// to row signs as a Householder QR of the whole block, since R^T R = Y^T Y).
//
// One workgroup per (block, chunk): rows [c CH, min((c + 1) CH, mrows)) of block blk's
// column-major matrix Y + blk * bstride (ld ldy, ell columns).  Thread t holds row t in
// LDS.  Step j: the column norm by a wavefront reduction, the reflector v, the products
// d_col = tau v^T A[:, col] for every later column at once (four row groups, then a sum
// over the groups), and the rank-one update of every row.  A column that is already zero
// needs no reflection.  R (ell x ell, rows past the chunk's row count zero) is written to
// rows c ell .. c ell + ell - 1 of Rout + blk * rstride (ld ldr).
template <int CH, int ELLM>
__global__ void __launch_bounds__(CH) k_qr_chunk(const double* Y, long ldy, long bstride, long mrows, int nch,
                                                 double* Rout, long ldr, long rstride, int ell) {
  constexpr int G = CH / 64;
  constexpr int LDA = ELLM + 1;
  __shared__ double A[CH * LDA];   // row t at A + t LDA
  __shared__ double V[CH];
  __shared__ double D[ELLM];
  __shared__ double part[G * ELLM];
  const int blk = blockIdx.x / nch, c = blockIdx.x % nch;
  const long row0 = (long)c * CH;
  const int m = (int)min((long)CH, mrows - row0);
  const double* Yb = Y + blk * bstride + row0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int col = 0; col < ell; ++col) A[tid * LDA + col] = (tid < m) ? Yb[tid + col * ldy] : 0.0;
  __syncthreads();
  const int jmax = min(m, ell);
  for (int j = 0; j < jmax; ++j) {
    const double x = (tid >= j && tid < m) ? A[tid * LDA + j] : 0.0;
    double s = x * x;
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) part[wave] = s;
    __syncthreads();
    s = 0.0;
    for (int g = 0; g < G; ++g) s += part[g];
    const double alpha = A[j * LDA + j];
    const double nx = sqrt(s);
    if (nx == 0.0) {   // the same for every thread: no reflection, row j of R is row j of A
      __syncthreads();
      continue;
    }
    const double sg = (alpha >= 0.0) ? 1.0 : -1.0;
    const double v0 = alpha + sg * nx;
    const double tau = 2.0 / (s - alpha * alpha + v0 * v0);
    V[tid] = (tid > j && tid < m) ? x : (tid == j ? v0 : 0.0);
    __syncthreads();
    for (int col = j + 1 + lane; col < ell; col += 64) {
      double d = 0.0;
      for (int t = j + wave; t < m; t += G) d += V[t] * A[t * LDA + col];
      part[wave * ELLM + col] = d;
    }
    __syncthreads();
    for (int col = j + 1 + tid; col < ell; col += CH) {
      double d = 0.0;
      for (int g = 0; g < G; ++g) d += part[g * ELLM + col];
      D[col] = tau * d;
    }
    __syncthreads();
    if (tid >= j && tid < m) {
      const double vt = V[tid];
      for (int col = j + 1; col < ell; ++col) A[tid * LDA + col] -= D[col] * vt;
      if (tid == j) A[j * LDA + j] = -sg * nx;
    }
    __syncthreads();
  }
  double* Rb = Rout + blk * rstride + (long)c * ell;
  for (int e = tid; e < ell * ell; e += CH) {
    const int i = e % ell, col = e / ell;
    Rb[i + (long)col * ldr] = (i <= col && i < jmax) ? A[i * LDA + col] : 0.0;
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
// stride ell*kc), sorted singular values sig (ell per block), kept ranks k.  One
// workgroup per block: each forms the level's factors d_j (a sum over the nb blocks)
// and scales its own block.
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
  double* Vb = V + (long)blockIdx.x * ell * kc;
  for (int e = threadIdx.x; e < ell * kc; e += blockDim.x) Vb[e] *= d[e / ell];
}

// Rows of the sample factored per chunk (at least 2 ell, so that every round at least
// halves the number of chunks: two stacked R factors fit one chunk) and the scratch the
// stacked R factors need (two halves of qr_stack_doubles each).
static int qr_chunk_rows(int ell) { return ell <= 72 ? 256 : 192; }
size_t qr_stack_doubles(int n, int nint, int ell) {
  return ((size_t)n / 2 / 128 + (size_t)nint + 1) * ell * ell;
}

hm_status sketch_compress(Model* m, const double* Y, int ldy, int ell, int l, int rank, double tol, double* S,
                          double* R, double* V, int kc, int* d_k, double* d_sig) {
  if (ell > ELLMAX) {
    set_error("rank + oversample exceeds 80");
    return HM_E_INVAL;
  }
  const int nb = 1 << (l - 1);
  // R of each block's left-child rows (block pi: rows 2 pi mrows .. 2 pi mrows + mrows)
  const int CH = qr_chunk_rows(ell);
  const size_t half = qr_stack_doubles(m->n, (1 << m->levels) - 1, ell);
  const double* src = Y;
  long rows = m->n >> l, bstride = 2 * rows, ld = ldy;
  for (int round = 0;; ++round) {
    if (round >= 64 || 2 * ell > CH) {
      set_error("sketch QR: the chunk rounds do not converge");
      return HM_E_INVAL;
    }
    const int nch = (int)((rows + CH - 1) / CH);
    double* dst;
    long ldr, rstride;
    if (nch == 1) {
      dst = R;
      ldr = ell;
      rstride = (long)ell * ell;
    } else {
      dst = S + (round & 1) * half;
      ldr = (long)nch * ell;
      rstride = ldr * ell;
      if ((size_t)nb * rstride > half) {
        set_error("sketch QR: stack scratch too small");
        return HM_E_INVAL;
      }
    }
    if (CH == 256)
      hipLaunchKernelGGL((k_qr_chunk<256, 72>), dim3(nb * nch), dim3(256), 0, m->stream, src, ld, bstride, rows, nch,
                         dst, ldr, rstride, ell);
    else
      hipLaunchKernelGGL((k_qr_chunk<192, 80>), dim3(nb * nch), dim3(192), 0, m->stream, src, ld, bstride, rows, nch,
                         dst, ldr, rstride, ell);
    HM_LAUNCH_CHECK();
    if (nch == 1) break;
    src = dst;
    ld = ldr;
    bstride = rstride;
    rows = (long)nch * ell;
  }
  hipLaunchKernelGGL(k_jacobi_svd, dim3(nb), dim3(256), 0, m->stream, R, ell, rank, tol, V, kc, d_k, d_sig,
                     m->d_flags);
  HM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_level_scale, dim3(nb), dim3(64), 0, m->stream, V, d_sig, d_k, nb, ell, kc);
  HM_LAUNCH_CHECK();
  return HM_OK;
}

}  // namespace hm
