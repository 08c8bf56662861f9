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
#include "gemm_core.h"
#include "wave_ops.h"

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

// X[l] -= f b[l] for l = l0..KP-1 (b in LDS, the same for every lane).  The reads of a
// range are all issued before its first multiply-add (the empty asm takes each value),
// so one LDS latency is paid per range rather than per pair of entries; KP = 64 runs
// as two ranges to stay within the register file.
template <int KP>
__device__ __forceinline__ void axpy_row_batched(double (&X)[KP], const double* b, double f, int l0) {
  constexpr int SP = KP > 48 ? KP / 2 : KP;
  double c[KP];
  const int l1 = l0 > SP ? l0 : SP;
#pragma unroll
  for (int l = l0; l < SP; ++l) c[l] = b[l];
#pragma unroll
  for (int l = l0; l < SP; ++l) asm volatile("" : "+v"(c[l]));
#pragma unroll
  for (int l = l0; l < SP; ++l) X[l] -= f * c[l];
#pragma unroll
  for (int l = l1; l < KP; ++l) c[l] = b[l];
#pragma unroll
  for (int l = l1; l < KP; ++l) asm volatile("" : "+v"(c[l]));
#pragma unroll
  for (int l = l1; l < KP; ++l) X[l] -= f * c[l];
#pragma unroll
  for (int l = l0; l < KP; ++l) asm volatile("" : "+v"(X[l]));
}

// ---------------------------------------------------------------------------
// Cholesky + triangular inverse of G (k x k, ld k), one node per workgroup of two
// wavefronts.  shift: if nonzero, G + s I with s = 11 (m k + k (k+1)) u ||.||_F^2,
// m = rows of the sketched block (shifted Cholesky-QR of Fukaya et al.);
// ||Y||_F^2 = tr(G).  Zero columns (k_P < k) are kept as identity so padding stays
// exactly zero.
//
// Right-looking Cholesky fused with the forward elimination of L Y = I.  With
// d_j = A(j, j) after step j - 1, f_ij = A(i, j) / d_j and l_ij = A(i, j) / sqrt(d_j),
// step j does
//   A(i, l) -= f_ij A(l, j)          (j < l <= i)
//   Y(i, c) -= f_ij Y(j, c)          (i > j)
// and L^{-1}(i, c) = Y(i, c) / sqrt(d_i).  Lane x of wavefront 0 holds row x of A, lane
// x of wavefront 1 column x of Y, in registers (KP >= k entries; rows and columns
// k..KP-1 an identity block that changes nothing).  Step j broadcasts column j of A
// through LDS; the rows' wavefront forms the multipliers f_xj and publishes them, and
// the Y wavefront applies step j one barrier later, so each wavefront's step is one
// broadcast read and one fused multiply-add per entry.  The rows' wavefront updates the
// whole row: entries right of the diagonal never feed an entry on or left of it (the
// update of A(i, l), l <= i, reads A(i, j) and A(l, j) with j < l), so they may hold
// anything and are not written out.  A pivot that is not positive is flagged and
// taken as 1.  R is staged through LDS so that its columns leave as contiguous stores.
// ---------------------------------------------------------------------------
template <int KP>
__global__ void __launch_bounds__(128) k_chol_inv(const double* G, long gstride, double* R, double* Rinv,
                                                  long rstride, int k, const int* kblk, int heap0, int hstep,
                                                  int shift, long mrows, int* flags) {
  constexpr int LDR = KP + 1;
  __shared__ double colj[2][64];   // column j of A
  __shared__ double fj[2][64];     // multipliers f_xj of step j
  __shared__ double sqd[64];       // sqrt(d_x)
  __shared__ double Rs[KP * LDR];  // R(i, x) at i + x LDR
  const int node = heap0 + blockIdx.x * hstep;
  // kept rank of the block whose left child is this node (kblk indexed by parent)
  const int kp = kblk ? kblk[(node - 1) >> 1] : k;
  const double* g = G + node * gstride;
  const int lane = threadIdx.x & 63;
  const bool rows = threadIdx.x < 64;   // wavefront 0: rows of A; wavefront 1: columns of Y
  const bool real = lane < kp;
  double s = 0.0;
  if (shift && rows) {
    double t = real ? g[lane + (long)lane * k] : 0.0;
    for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
    s = 11.0 * ((double)mrows * kp + (double)kp * (kp + 1)) * 1.1102230246251565e-16 * t;
  }
  double X[KP];
#pragma unroll
  for (int l = 0; l < KP; ++l) {
    double v;
    if (rows) {
      v = (real && l < kp) ? g[lane + (long)l * k] : (lane == l ? 1.0 : 0.0);
      if (real && l == lane) v += s;
    } else {
      v = (l == lane) ? 1.0 : 0.0;
    }
    X[l] = v;
  }
  double myd = 1.0;
  bool bad = false;
  // the two wavefronts run their own copy of the step loop (the same barriers), so
  // that each step's broadcast reads form one straight run of code
  if (rows) {
#pragma unroll
    for (int j = 0; j < KP; ++j) {
      double* cb = colj[j & 1];
      cb[lane] = X[j];
      __syncthreads();
      double d = cb[j];
      if (!(d > 0.0)) {
        bad = true;
        d = 1.0;
      }
      if (lane == j) myd = d;
      const double f = X[j] * (1.0 / d);
      fj[j & 1][lane] = f;
      axpy_row_batched<KP>(X, cb, f, j + 1);
    }
  } else {
#pragma unroll
    for (int j = 0; j < KP; ++j) {
      __syncthreads();
      if (j > 0) {   // step j - 1, its multipliers published before this barrier
        const double y = X[j - 1];
        axpy_row_batched<KP>(X, fj[(j - 1) & 1], y, j);
      }
    }
    // step KP - 1 updates no entry
  }
  if (bad && threadIdx.x == 0) atomicOr(flags, (int)DF_QR_FAIL);
  if (rows) sqd[lane] = sqrt(myd);
  __syncthreads();
  if (rows) {
    // R = L^T (upper): column x of R is row x of L, held by lane x
    const double sx = sqrt(myd);
#pragma unroll
    for (int i = 0; i < KP; ++i)
      if (lane < KP) Rs[i + lane * LDR] = (i < lane) ? X[i] / sqd[i] : (i == lane ? sx : 0.0);
  } else if (lane < k) {
    // Rinv = (L^{-1})^T: Rinv(i, j) = Y(j, i) / sqrt(d_j) for j >= i; row i held by lane i
    double* Ri = Rinv + node * rstride + lane;
#pragma unroll
    for (int j = 0; j < KP; ++j)
      if (j < k) Ri[(long)j * k] = (j >= lane) ? X[j] / sqd[j] : 0.0;
  }
  __syncthreads();
  double* Ro = R + node * rstride;
  for (int e = threadIdx.x; e < k * k; e += 128) {
    const int i = e % k, x = e / k;
    Ro[e] = Rs[i + x * LDR];
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
//
// One node per workgroup of four wavefronts.  The k x k products run on the FP64
// matrix cores from LDS (leading dimension KP + 1, odd, so that column reads hit
// distinct banks); k..KP-1 is a zero border of S_a and S_b, i.e. an identity block of
// Sig that pivots on itself and changes nothing.
// ---------------------------------------------------------------------------
// C tile (ti, tj) of A B (KP x KP, ld LD, in LDS) into a 16 x 16 accumulator:
// element v of lane l is C(16 ti + 4 v + l / 16, 16 tj + l % 16)
template <int KP>
__device__ __forceinline__ hm_v4d node_mm_tile(const double* A, const double* B, int ti, int tj, int lane) {
  constexpr int LD = KP + 1;
  const int li = lane & 15, lk = lane >> 4;
  hm_v4d acc = MfmaPrec<0>::zero();
#pragma unroll
  for (int kk = 0; kk < KP; kk += 4)
    acc = MfmaPrec<0>::mfma(A[(16 * ti + li) + (kk + lk) * LD], B[(kk + lk) + (16 * tj + li) * LD], acc);
  return acc;
}

template <int KP>
__global__ void __launch_bounds__(256) k_node_lu(const double* S, long sstride, double* Nout, long nstride,
                                                 double* logdet, int k, int heap0, int* flags) {
  constexpr int LD = KP + 1, NT = KP / 16;
  __shared__ double Sa[KP * LD];
  __shared__ double Sb[KP * LD];
  __shared__ double Sg[KP * LD];   // Sig, then Sig^{-1}
  __shared__ double Si[KP * LD];   // the accumulated row operations, then S_b Sig^{-1}
  __shared__ double mul[2][64];
  __shared__ double prow[2][64];   // pivot row of wavefront 0 (Sig) and 1 (row operations)
  __shared__ int piv[64];
  __shared__ double pval[64];
  const int P = heap0 + blockIdx.x;
  const int a = 2 * P + 1, b = 2 * P + 2;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int e = tid; e < KP * KP; e += 256) {
    const int i = e % KP, j = e / KP;
    const bool in = i < k && j < k;
    Sa[i + j * LD] = in ? S[a * sstride + i + (long)j * k] : 0.0;
    Sb[i + j * LD] = in ? S[b * sstride + i + (long)j * k] : 0.0;
  }
  __syncthreads();
  const int li = lane & 15, lk = lane >> 4;
  // Sig = I - S_a S_b
  for (int t = wave; t < NT * NT; t += 4) {
    const int ti = t % NT, tj = t / NT;
    const hm_v4d acc = node_mm_tile<KP>(Sa, Sb, ti, tj, lane);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * ti + 4 * v + lk, c = 16 * tj + li;
      Sg[r + c * LD] = (r == c ? 1.0 : 0.0) - acc[v];
    }
  }
  __syncthreads();
  // Gauss-Jordan elimination with partial pivoting on [Sig | I]: lane i of wavefront 0
  // holds row i of Sig, lane i of wavefront 1 row i of the row operations Y.  Step j:
  // wavefront 0 finds the pivot p_j (the largest |Sig(i, j)| over rows not yet used,
  // ties to the lower row) and the multipliers Sig(i, j) / Sig(p_j, j); every other
  // row subtracts its multiple of row p_j, broadcast through LDS by its owner.  Then
  // Sig^{-1}(j, :) = Y(p_j, :) / Sig(p_j, j) and det Sig = sign(pivot permutation) *
  // prod_j Sig(p_j, j).
  // Wavefront 0 keeps only the columns not yet eliminated, shifted so that X[0] is
  // column j at step j (every register index stays a constant).
  double X[KP];
#pragma unroll
  for (int c = 0; c < KP; ++c) X[c] = (wave == 0 && lane < KP) ? Sg[lane + c * LD] : (lane == c ? 1.0 : 0.0);
  bool used = lane >= KP;
#pragma unroll 1
  for (int j = 0; j < KP; ++j) {
    if (wave == 0) {
      double best = -1.0;
      int bi = 64;
      if (!used) {
        best = fabs(X[0]);
        if (!(best <= INFINITY)) best = INFINITY;   // NaN ranks first: the order stays total
        bi = lane;
      }
      const int p = __builtin_amdgcn_readfirstlane(wave_argmax(best, bi));
      const double pv = readlane_d(X[0], p);
      const double rp = (pv != 0.0) ? 1.0 / pv : 0.0;
      mul[j & 1][lane] = (lane != p) ? X[0] * rp : 0.0;
      if (lane == p) used = true;
      if (lane == 0) {
        piv[j] = p;
        pval[j] = pv;
      }
    }
    __syncthreads();
    if (wave < 2) {
      const int p = piv[j];
      const double f = mul[j & 1][lane];   // 0 on the pivot row
      double* rb = prow[wave];
      if (lane == p) {
#pragma unroll
        for (int c = 0; c < KP; ++c) rb[c] = X[c];
      }
      // the pivot lane's stores are ordered before every lane's reads (a wavefront-scope
      // release and acquire: without them the compiler may hoist the other lanes' reads
      // above the stores, as it sees no dependence between lanes)
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // the pivot row's entries are all read before the first multiply-add (the empty
      // asm takes each value), so one LDS latency is paid per half row
      constexpr int SP = KP > 32 ? KP / 2 : KP;
      double c_[KP];
#pragma unroll
      for (int c = 0; c < SP; ++c) c_[c] = rb[c];
#pragma unroll
      for (int c = 0; c < SP; ++c) asm volatile("" : "+v"(c_[c]));
#pragma unroll
      for (int c = SP; c < KP; ++c) c_[c] = rb[c];
      if (wave == 0) {
        // columns j+1.. (X[1..]) minus f times the pivot row's, shifted down by one
#pragma unroll
        for (int c = 0; c + 1 < SP; ++c) X[c] = X[c + 1] - f * c_[c + 1];
#pragma unroll
        for (int c = SP; c < KP; ++c) asm volatile("" : "+v"(c_[c]));
#pragma unroll
        for (int c = SP - 1; c + 1 < KP; ++c) X[c] = X[c + 1] - f * c_[c + 1];
        X[KP - 1] = 0.0;
      } else {
#pragma unroll
        for (int c = 0; c < SP; ++c) X[c] -= f * c_[c];
#pragma unroll
        for (int c = SP; c < KP; ++c) asm volatile("" : "+v"(c_[c]));
#pragma unroll
        for (int c = SP; c < KP; ++c) X[c] -= f * c_[c];
      }
#pragma unroll
      for (int c = 0; c < KP; ++c) asm volatile("" : "+v"(X[c]));
    }
  }
  // Y rows into LDS; then Sig^{-1}(j, c) = Y(p_j, c) / Sig(p_j, j) into Sg
  if (wave == 1 && lane < KP) {
#pragma unroll
    for (int c = 0; c < KP; ++c) Si[lane + c * LD] = X[c];
  }
  __syncthreads();
  for (int e = tid; e < KP * KP; e += 256) {
    const int j = e % KP, c = e / KP;
    Sg[j + c * LD] = Si[piv[j] + c * LD] / pval[j];
  }
  if (wave == 3) {
    // log |det| and the sign: pivot signs times the parity of the pivot permutation
    // (its inversion count), over the first k steps (the border pivots on itself)
    double ls = 0.0;
    int odd = 0;
    if (lane < k) {
      ls = log(fabs(pval[lane]));
      int inv = pval[lane] < 0.0 ? 1 : 0;
      const int pl = piv[lane];
      for (int q = lane + 1; q < k; ++q) inv += piv[q] < pl ? 1 : 0;
      odd = inv & 1;
    }
    for (int off = 32; off > 0; off >>= 1) {
      ls += __shfl_xor(ls, off, 64);
      odd ^= __shfl_xor(odd, off, 64);
    }
    if (lane == 0) {
      logdet[P] = ls;
      if (odd || !isfinite(ls)) atomicOr(flags, (int)DF_NOT_SPD_NODE);
    }
  }
  __syncthreads();
  // P1 = S_b Sig^{-1} -> Si (the row operations are no longer needed)
  for (int t = wave; t < NT * NT; t += 4) {
    const int ti = t % NT, tj = t / NT;
    const hm_v4d acc = node_mm_tile<KP>(Sb, Sg, ti, tj, lane);
#pragma unroll
    for (int v = 0; v < 4; ++v) Si[(16 * ti + 4 * v + lk) + (16 * tj + li) * LD] = acc[v];
  }
  __syncthreads();
  const int m = 2 * k;
  double* No = Nout + P * nstride;
  for (int e = tid; e < k * k; e += 256) {
    const int i = e % k, j = e / k;
    No[i + (long)j * m] = -Si[i + j * LD];          // N11 = -S_b Sig^{-1}
    No[(k + i) + (long)j * m] = Sg[i + j * LD];     // N21 = Sig^{-1}
  }
  for (int t = wave; t < 2 * NT * NT; t += 4) {
    const int which = t / (NT * NT), tt = t % (NT * NT);
    const int ti = tt % NT, tj = tt / NT;
    // which 0: N12 = I + P1 S_a;  which 1: N22 = -Sig^{-1} S_a
    const hm_v4d acc = node_mm_tile<KP>(which ? Sg : Si, Sa, ti, tj, lane);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 16 * ti + 4 * v + lk, j = 16 * tj + li;
      if (i < k && j < k) {
        if (which) No[(k + i) + (long)(k + j) * m] = -acc[v];
        else No[i + (long)(k + j) * m] = (i == j ? 1.0 : 0.0) + acc[v];
      }
    }
  }
}

hm_status chol_inv_nodes(Model* m, const double* G, long gstride, double* R, double* Rinv, long rstride,
                         int k, const int* d_kblk, int heap0, int hstep, int cnt, int shift, long mrows) {
  if (k > KMAX) {
    set_error("panel width exceeds the per-node LDS limit (64)");
    return HM_E_INVAL;
  }
  if (k <= 16)
    hipLaunchKernelGGL(k_chol_inv<16>, dim3(cnt), dim3(128), 0, m->stream, G, gstride, R, Rinv, rstride, k, d_kblk,
                       heap0, hstep, shift, mrows, m->d_flags);
  else if (k <= 32)
    hipLaunchKernelGGL(k_chol_inv<32>, dim3(cnt), dim3(128), 0, m->stream, G, gstride, R, Rinv, rstride, k, d_kblk,
                       heap0, hstep, shift, mrows, m->d_flags);
  else if (k <= 48)
    hipLaunchKernelGGL(k_chol_inv<48>, dim3(cnt), dim3(128), 0, m->stream, G, gstride, R, Rinv, rstride, k, d_kblk,
                       heap0, hstep, shift, mrows, m->d_flags);
  else
    hipLaunchKernelGGL(k_chol_inv<64>, dim3(cnt), dim3(128), 0, m->stream, G, gstride, R, Rinv, rstride, k, d_kblk,
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
  if (k <= 16)
    hipLaunchKernelGGL(k_node_lu<16>, dim3(cnt), dim3(256), 0, m->stream, S, sstride, Nout, nstride, logdet, k,
                       heap0, m->d_flags);
  else if (k <= 32)
    hipLaunchKernelGGL(k_node_lu<32>, dim3(cnt), dim3(256), 0, m->stream, S, sstride, Nout, nstride, logdet, k,
                       heap0, m->d_flags);
  else if (k <= 48)
    hipLaunchKernelGGL(k_node_lu<48>, dim3(cnt), dim3(256), 0, m->stream, S, sstride, Nout, nstride, logdet, k,
                       heap0, m->d_flags);
  else
    hipLaunchKernelGGL(k_node_lu<64>, dim3(cnt), dim3(256), 0, m->stream, S, sstride, Nout, nstride, logdet, k,
                       heap0, m->d_flags);
  HM_LAUNCH_CHECK();
  return HM_OK;
}

}  // namespace hm
