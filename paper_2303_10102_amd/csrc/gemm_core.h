// FP64 tile-GEMM core shared by all panel/leaf/transform kernels.
//
// A workgroup of NT = (BM/TM)*(BN/TN) threads computes a BM x BN tile of
// C = sum_k A(i,k) B(k,j).  Operands are fetched through loader functors so the
// same core serves plain column-major GEMMs, per-leaf panel products with tree
// addressing, and the sine transform with the tree<->grid gather fused into the
// load.  Tiles are staged through LDS; each thread keeps a TM x TN register
// tile whose rows/columns are strided by BM/TM and BN/TN (conflict-free LDS
// reads for 8-byte elements).
#pragma once
#include <hip/hip_runtime.h>

namespace hm {

template <int BM, int BN, int BK, int TM, int TN>
struct TileCfg {
  static constexpr int NT = (BM / TM) * (BN / TN);
  static constexpr int RS = BM / TM;   // row stride of a thread's register tile
  static constexpr int CS = BN / TN;   // column stride
  static constexpr int LDS_A = BK * (BM + 1);
  static constexpr int LDS_B = BK * (BN + 1);
  static constexpr int LDS_DOUBLES = LDS_A + LDS_B;
};

// LA: double operator()(int i, int k) const  -- i in [0,BM) tile row, k global
//     static constexpr bool kfast            -- consecutive k adjacent in memory
// LB: double operator()(int k, int j) const  -- j in [0,BN) tile column
template <int BM, int BN, int BK, int TM, int TN, class LA, class LB>
__device__ __forceinline__ void tile_gemm_acc(const LA& la, const LB& lb, int k0, int k1,
                                              double (&acc)[TM][TN], double* smem) {
  using C = TileCfg<BM, BN, BK, TM, TN>;
  double* As = smem;             // [BK][BM+1]
  double* Bs = smem + C::LDS_A;  // [BK][BN+1]
  const int tid = threadIdx.x;
  const int tr = tid / C::CS;
  const int tc = tid % C::CS;
  for (int kb = k0; kb < k1; kb += BK) {
    // ---- stage A tile
#pragma unroll
    for (int e0 = 0; e0 < BM * BK; e0 += C::NT) {
      int e = e0 + tid;
      int i, kk;
      if (LA::kfast) { kk = e % BK; i = e / BK; } else { i = e % BM; kk = e / BM; }
      int k = kb + kk;
      As[kk * (BM + 1) + i] = (k < k1) ? la(i, k) : 0.0;
    }
    // ---- stage B tile
#pragma unroll
    for (int e0 = 0; e0 < BN * BK; e0 += C::NT) {
      int e = e0 + tid;
      int j, kk;
      if (LB::kfast) { kk = e % BK; j = e / BK; } else { j = e % BN; kk = e / BN; }
      int k = kb + kk;
      Bs[kk * (BN + 1) + j] = (k < k1) ? lb(k, j) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; ++kk) {
      double a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) a[i] = As[kk * (BM + 1) + tr + i * C::RS];
#pragma unroll
      for (int j = 0; j < TN; ++j) b[j] = Bs[kk * (BN + 1) + tc + j * C::CS];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
}

template <int BM, int BN, int TM, int TN>
__device__ __forceinline__ void tile_zero(double (&acc)[TM][TN]) {
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = 0.0;
}

// ST: void operator()(int i, int j, double v) const  (tile-relative; does its own bounds)
template <int BM, int BN, int BK, int TM, int TN, class ST>
__device__ __forceinline__ void tile_store(const ST& st, const double (&acc)[TM][TN]) {
  using C = TileCfg<BM, BN, BK, TM, TN>;
  const int tid = threadIdx.x;
  const int tr = tid / C::CS;
  const int tc = tid % C::CS;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) st(tr + i * C::RS, tc + j * C::CS, acc[i][j]);
}

// Standard configuration used by the panel kernels.
constexpr int GBM = 64, GBN = 64, GBK = 16, GTM = 4, GTN = 4;
using GCfg = TileCfg<GBM, GBN, GBK, GTM, GTN>;

}  // namespace hm
