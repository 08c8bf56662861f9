// Leaf blocks: extraction from the stacked-identity sample, Cholesky, log-det,
// explicit inverses.
//
// The leaf blocks of K~ are read from (K - sum_l H_l) [I; I; ...] (Sec. 3.2,
// eq. "leaf sample") and symmetrised.  The factorisation K~ = Dbar * prod(I + U V^T)
// starts by factoring out the block-diagonal Dbar of leaf blocks (App. C, eq.
// "factor out leaf"); its log-determinant is 2 sum log diag(chol(D_L)).
#include <cmath>

#include "hm_internal.h"

namespace hm {

// D_L = (Z_L + Z_L^T)/2 with Z rows in tree order (ld ldz), leaf-major output.
__global__ void k_leaf_sym(const double* Z, int ldz, double* D, int nl, double scale) {
  const int L = blockIdx.y;
  const long r0 = (long)L * nl;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nl * nl) return;
  const int i = e % nl, j = e / nl;
  const double a = Z[r0 + i + (long)j * ldz], b = Z[r0 + j + (long)i * ldz];
  D[(long)L * nl * nl + e] = 0.5 * scale * (a + b);
}

hm_status leaf_sym(Model* m, const double* Z, int ldz, double* D) {
  const int nl = m->nl;
  hipLaunchKernelGGL(k_leaf_sym, dim3(ceil_div(nl * nl, 256), m->nleaves), dim3(256), 0, m->stream, Z, ldz, D, nl,
                     1.0);
  HM_LAUNCH_CHECK();
  return HM_OK;
}

constexpr int CNB = 32;      // Cholesky block width
constexpr int NLMAX = 512;   // largest leaf handled

// In-place blocked Cholesky (lower) of W (nl x nl, column-major), one leaf per
// workgroup.  logdet[L] = 2 sum log L_ii.  A non-positive pivot sets a flag and
// is replaced by 1 so the kernel still completes.
__global__ void __launch_bounds__(256) k_leaf_chol(double* W, int nl, double* logdet, int* flags) {
  __shared__ double panel[NLMAX * CNB];  // rows jb..nl-1 of the current block column
  const int L = blockIdx.x;
  double* A = W + (long)L * nl * nl;
  const int tid = threadIdx.x, nt = blockDim.x;
  double lsum = 0.0;  // accumulated by thread 0
  int bad = 0;
  for (int jb = 0; jb < nl; jb += CNB) {
    const int nb = min(CNB, nl - jb);
    const int rows = nl - jb;
    // stage the block column (rows jb..nl-1, cols jb..jb+nb-1) into LDS, row-major in t
    for (int e = tid; e < rows * nb; e += nt) {
      int i = e % rows, t = e / rows;
      panel[i * CNB + t] = A[(jb + i) + (long)(jb + t) * nl];
    }
    __syncthreads();
    // unblocked factorisation of the diagonal block + triangular solve of the rest:
    for (int t = 0; t < nb; ++t) {
      if (tid == 0) {
        double d = panel[t * CNB + t];
        if (!(d > 0.0)) { bad = 1; d = 1.0; }
        d = sqrt(d);
        panel[t * CNB + t] = d;
        lsum += 2.0 * log(d);
      }
      __syncthreads();
      const double piv = panel[t * CNB + t];
      for (int i = t + 1 + tid; i < rows; i += nt) panel[i * CNB + t] /= piv;
      __syncthreads();
      // update columns t+1..nb-1 of the block column
      for (int e = tid; e < (rows - t - 1) * (nb - t - 1); e += nt) {
        int i = t + 1 + e % (rows - t - 1), u = t + 1 + e / (rows - t - 1);
        if (i >= u) panel[i * CNB + u] -= panel[i * CNB + t] * panel[u * CNB + t];
      }
      __syncthreads();
    }
    // write back the factored block column (lower part)
    for (int e = tid; e < rows * nb; e += nt) {
      int i = e % rows, t = e / rows;
      A[(jb + i) + (long)(jb + t) * nl] = (i >= t) ? panel[i * CNB + t] : 0.0;
    }
    // trailing update: A[i,l] -= sum_t P[i,t] P[l,t] for jb+nb <= l <= i
    const int r2 = nl - jb - nb;
    for (int e = tid; e < r2 * r2; e += nt) {
      int i = e % r2, l = e / r2;
      if (i < l) continue;
      double s = 0.0;
      const double* pi = panel + (nb + i) * CNB;
      const double* pl = panel + (nb + l) * CNB;
      for (int t = 0; t < nb; ++t) s += pi[t] * pl[t];
      A[(jb + nb + i) + (long)(jb + nb + l) * nl] -= s;
    }
    __syncthreads();
  }
  if (tid == 0) {
    logdet[L] = lsum;
    if (bad) atomicOr(flags, (int)DF_NOT_SPD_LEAF);
  }
}

// U = L^{-T} (upper, column-major), i.e. L^{-1} stored row-major: U[j + i*nl] = (L^{-1})(i, j).
// Blocked forward substitution on the identity, one leaf per workgroup.  For
// block row ib (rows r0..r0+nb): R = E - L[r0:, 0:r0] X[0:r0, :], X[r0:, :] = L_ii^{-1} R.
// Thread j owns column j; the block row of L is staged in LDS (read as
// broadcasts), earlier rows of X are read back from U (coalesced over j).
constexpr int TB = 32;
__global__ void __launch_bounds__(256) k_leaf_trinv(const double* Lf, double* U, int nl) {
  __shared__ double Lp[TB * NLMAX];   // Lp[r * nl + c] = L(r0 + r, c), c < r0 + nb
  __shared__ double Ti[TB * TB];      // (L_ii)^{-1}, row-major
  const int Lidx = blockIdx.x;
  const double* A = Lf + (long)Lidx * nl * nl;
  double* X = U + (long)Lidx * nl * nl;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int r0 = 0; r0 < nl; r0 += TB) {
    const int nb = min(TB, nl - r0);
    const int w = r0 + nb;
    for (int e = tid; e < nb * w; e += nt) {
      int r = e / w, c = e % w;
      Lp[r * nl + c] = A[(r0 + r) + (long)c * nl];
    }
    __syncthreads();
    // inverse of the diagonal block: column t of Ti^T ... thread t solves L_ii x = e_t
    if (tid < nb) {
      const int t = tid;
      for (int r = 0; r < nb; ++r) {
        double v = (r == t) ? 1.0 : 0.0;
        for (int q = t; q < r; ++q) v -= Lp[r * nl + r0 + q] * Ti[q * TB + t];
        Ti[r * TB + t] = (r < t) ? 0.0 : v / Lp[r * nl + r0 + r];
      }
    }
    __syncthreads();
    for (int j = tid; j < nl; j += nt) {
      double acc[TB];
#pragma unroll
      for (int r = 0; r < TB; ++r) acc[r] = (r < nb && r0 + r == j) ? 1.0 : 0.0;
      if (j < r0) {
        // columns c in [j, r0): batches of 8 independent loads, then the updates
        for (int c0 = j; c0 < r0; c0 += 8) {
          double xr[8];
#pragma unroll
          for (int t = 0; t < 8; ++t) xr[t] = (c0 + t < r0) ? X[j + (long)(c0 + t) * nl] : 0.0;
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            const int c = min(c0 + t, r0 - 1);
#pragma unroll
            for (int r = 0; r < TB; ++r)
              if (r < nb) acc[r] -= Lp[r * nl + c] * xr[t];
          }
        }
      }
#pragma unroll
      for (int r = 0; r < TB; ++r) {
        if (r >= nb) break;
        double v = 0.0;
        for (int t = 0; t < nb; ++t) v += Ti[r * TB + t] * acc[t];
        X[j + (long)(r0 + r) * nl] = (j <= r0 + r) ? v : 0.0;
      }
    }
    __syncthreads();
  }
}

// Dinv_L = L^{-T} L^{-1};  logdet_leaf[L] = log det D_L.  work: nleaves*nl*nl doubles.
hm_status leaf_factor(Model* m, const double* D, double* Dinv, double* logdet_leaf, double* work) {
  const int nl = m->nl;
  if (nl > NLMAX) {
    set_error("leaf size exceeds 512");
    return HM_E_INVAL;
  }
  const long sz = (long)m->nleaves * nl * nl;
  HM_HIP(hipMemcpyAsync(work, D, sz * sizeof(double), hipMemcpyDeviceToDevice, m->stream));
  hipLaunchKernelGGL(k_leaf_chol, dim3(m->nleaves), dim3(256), 0, m->stream, work, nl, logdet_leaf, m->d_flags);
  HM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_leaf_trinv, dim3(m->nleaves), dim3(256), 0, m->stream, work, Dinv, nl);
  HM_LAUNCH_CHECK();
  // Dinv currently holds U = L^{-T}; form U U^T = L^{-T} L^{-1} into work, then copy back
  HM_CHECK(gemm(m->stream, false, true, nl, nl, nl, 1.0, Dinv, nl, (long)nl * nl, Dinv, nl, (long)nl * nl, 0.0,
                work, nl, (long)nl * nl, m->nleaves));
  HM_HIP(hipMemcpyAsync(Dinv, work, sz * sizeof(double), hipMemcpyDeviceToDevice, m->stream));
  return HM_OK;
}

}  // namespace hm
